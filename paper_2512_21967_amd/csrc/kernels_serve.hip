// Continuous-batching BFS server: one persistent launch serving requests of 1..64
// sources on up to four resident graphs.
//
// Each graph carries the state of the k-source BFS (kernels_multi.hip): a 64-bit
// (current, next) visited pair and a 64-bit frontier word per vertex, bit c for
// source column c, and a state byte per vertex.  All graphs advance together, one
// server iteration at a time; an iteration is one level of every running column:
// Stage 1 pulls over the concatenated VSS queues of all graphs (the Boolean SpMM
// of the stacked frontiers, Section 2, with Algorithm 3's lazy update), Stage 2
// folds the new bits of every graph into levels, frontier words and the next
// queues.  Columns start at different iterations: a column admitted at iteration
// a writes level i - a + 1 for the bits it gains in iteration i.
//
// At the start of every iteration one wavefront of workgroup 0 runs the control
// step while the other wavefronts run Stage 1 (so an iteration costs two grid
// barriers); its admissions take effect at the level boundary after Stage 2, and
// the admitted columns start with the next iteration:
//   * columns that gained no bit in the last iteration are finished; a request
//     whose columns have all finished is reported done in its mailbox slot (host
//     memory), after a system-scope release so that its levels are visible;
//   * newly published requests are copied from the mailbox ring, and waiting
//     requests are admitted, oldest first per graph, into free columns;
//   * with nothing running or waiting, it polls the mailbox until new work, a
//     stop request or the idle limit (then the launch ends; the host starts a new
//     one when requests arrive).
// Admitted columns are cleared (bits a finished column left behind) and their
// output rows initialised in two extra phases, and the VSS ranges of their
// sources' slice sets join the current queue.  Every wait is bounded: the grid
// barrier waits for co-resident workgroups only, and the idle poll ends at the
// idle limit.
#include <hip/hip_runtime.h>

#include "device_common.hpp"
#include "kernels.hpp"

namespace blest {
namespace {

constexpr uint64_t kDenseFrac = 1;  // dense Stage 2 only when the queue holds every VSS
constexpr uint32_t kStage2Rounds = 4;  // words per thread and pass of Stage 2

// A poll of a host-written word: a relaxed system-scope load reads memory without
// the cache invalidation an acquire at system scope costs; the control step issues
// one acquire fence only when a poll shows new tickets.
__device__ __forceinline__ uint32_t sys_poll(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ void sys_store(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ uint32_t* qlen_of(const ServeParams& p, uint32_t g, uint32_t r) {
  return p.ctrl + kQlen + (g * 3 + r) * kLine;
}
__device__ __forceinline__ uint32_t sorig(const ServeGraph& G, uint32_t u) { return G.orig_id ? G.orig_id[u] : u; }

__device__ __forceinline__ uint64_t wave_or64(uint64_t x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)x, o, kWave);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(x >> 32), o, kWave);
    x |= ((uint64_t)hi << 32) | lo;
  }
  return x;
}

__device__ __forceinline__ uint32_t wave_max(uint32_t x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x = max(x, (uint32_t)__shfl_xor((int)x, o, kWave));
  return x;
}

// Values of the control step live in device memory and are written by lane 0;
// every lane loads them through lane 0 so that the wavefront's control flow is
// uniform.
__device__ __forceinline__ uint32_t u32_of_lane0(const uint32_t* p) { return readlane(*p, 0); }
__device__ __forceinline__ uint64_t u64_of_lane0(const unsigned long long* p) { return readlane64(*p, 0); }

// ---- control step: one wavefront (workgroup 0, wavefront 0) ----
__device__ void serve_control(const ServeParams& p, uint32_t it) {
  ServeState* st = p.st;
  ServeMailbox* mb = p.mb;
  const uint32_t lane = lane_id();
  // 1. finished columns (no new bit in the last iteration); per request slot, the
  // running-column count and the deepest level are kept by lane 0
  uint64_t done_slots[kServeRing / 64] = {};
  // Every word this step reads from the state in the common case, loaded at once
  // (a chain of dependent loads costs a memory round trip each): lane 4j + g holds
  // active, admitted and alive of graph g for j = 0, 1, 2; lanes 12 and 13 the
  // ticket counters; and every lane its column's admission iteration per graph.
  // Only this wavefront writes active, admitted and the counters, and Stage 2's
  // ORs into alive are complete (they precede the grid barrier before this step).
  uint64_t wv = 0;
  if (lane < 12 && (lane & 3u) < p.ngraphs)
    wv = lane < 4 ? st->active[lane] : lane < 8 ? st->admitted[lane - 4] : st->alive[lane - 8];
  const uint32_t cw = lane == 12 ? st->seen : lane == 13 ? st->consumed : 0u;
  uint32_t cstart[kServeMaxGraphs];
#pragma unroll
  for (uint32_t g = 0; g < kServeMaxGraphs; ++g) cstart[g] = g < p.ngraphs ? st->col_start[g][lane] : 0u;
  uint64_t actv[kServeMaxGraphs];  // active columns per graph, kept current below
#pragma unroll
  for (uint32_t g = 0; g < kServeMaxGraphs; ++g) actv[g] = readlane64(wv, g);
  for (uint32_t g = 0; g < p.ngraphs; ++g) {
    const uint64_t act = actv[g];
    // a BFS has at most n + 1 levels: a column older than that is ended (a guard;
    // it never fires when Stage 2 reports growth correctly)
    const uint32_t n = g == 0 ? p.g[0].n : g == 1 ? p.g[1].n : g == 2 ? p.g[2].n : p.g[3].n;
    const uint32_t cs = g == 0 ? cstart[0] : g == 1 ? cstart[1] : g == 2 ? cstart[2] : cstart[3];
    const bool overdue = ((act >> lane) & 1ull) && it - cs > n + 2;
    // columns admitted by the previous control step start in this iteration: they
    // have not had a Stage 2 yet
    const uint64_t fresh = readlane64(wv, 4 + g);
    const uint64_t fin = act & ((~readlane64(wv, 8 + g) & ~fresh) | __ballot(overdue));
    if (!fin) continue;
    const bool mine = (fin >> lane) & 1ull;
    const uint32_t r = mine ? st->col_ticket[g][lane] % kServeRing : 0u;
    const uint32_t lev = mine ? it - st->col_start[g][lane] : 0u;  // levels of the column (0 included)
    uint64_t left = __ballot(mine);
    while (left) {
      const uint32_t lead = __ffsll((unsigned long long)left) - 1;
      const uint32_t rr = readlane(r, lead);
      const uint64_t grp = __ballot(mine && r == rr);
      const uint32_t lv = wave_max(mine && r == rr ? lev : 0u);
      if (lane == 0) {
        const uint32_t rem = st->remaining[rr] - (uint32_t)__popcll(grp);
        st->remaining[rr] = rem;
        st->maxlev[rr] = max(st->maxlev[rr], lv);
        if (rem == 0) done_slots[rr / 64] |= 1ull << (rr % 64);
      }
      left &= ~grp;
    }
    actv[g] = act & ~fin;
    if (lane == 0) {
      st->active[g] = actv[g];
      st->dirty[g] |= fin;
    }
  }
  // 2. report finished requests (lane 0): the levels, written by every workgroup
  // before the grid barrier that precedes this step, are made visible to the host
  // before the slot says done
  if (lane == 0) {
    bool any_done = false;
    for (int i = 0; i < (int)(kServeRing / 64); ++i) any_done |= done_slots[i] != 0;
    if (any_done) {
      __threadfence_system();
      for (int i = 0; i < (int)(kServeRing / 64); ++i) {
        uint64_t m = done_slots[i];
        while (m) {
          const uint32_t r = i * 64 + (__ffsll((unsigned long long)m) - 1);
          m &= m - 1;
          ServeSlot* hs = &mb->slot[r];
          hs->levels = st->maxlev[r];
          hs->done_iter = it;
          st->slot[r].state = 3;
          sys_store(&hs->state, 3u);
        }
      }
    }
    for (uint32_t g = 0; g < p.ngraphs; ++g) {
      st->alive[g] = 0;
      st->admitted[g] = 0;
    }
  }
  // 3. copy newly published requests; 4. admit; 5. idle wait.  stop == 2 (abort,
  // from the host) ends the launch at once, running columns or not.
  uint32_t n_admit = 0, exit_now = 0;
  const uint64_t t_idle0 = __builtin_amdgcn_s_memrealtime();
  uint32_t seen = readlane(cw, 12), consumed = readlane(cw, 13);
  for (;;) {
    // both polls are issued before either is used
    const uint32_t stop_w = sys_poll(&mb->stop), sub_w = sys_poll(&mb->submitted);
    if (readlane(stop_w, 0) == 2) {
      exit_now = 1;
      break;
    }
    const uint32_t sub = readlane(sub_w, 0);
    // the host publishes a slot before it raises `submitted`: order the slot reads
    // after the poll that saw it
    if (sub != seen) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
    for (uint32_t c = 0; c < 16 && seen != sub; ++c, ++seen) {
      const uint32_t r = seen % kServeRing;
      const uint32_t* src = reinterpret_cast<const uint32_t*>(&mb->slot[r]);
      uint32_t* dst = reinterpret_cast<uint32_t*>(&st->slot[r]);
      constexpr uint32_t kWords = sizeof(ServeSlot) / 4;
      for (uint32_t w = lane; w < kWords; w += kWave) dst[w] = src[w];
    }
    // the copies of all lanes are complete before any lane reads them
    __threadfence_block();
    __builtin_amdgcn_wave_barrier();
    if (lane == 0) st->seen = seen;
    // admission, oldest first; a graph whose oldest waiting request does not fit
    // admits nothing newer this time (per-graph first-come order)
    uint32_t blocked = 0;
    for (uint32_t t = consumed; t != seen; ++t) {
      const uint32_t r = t % kServeRing;
      ServeSlot* ds = &st->slot[r];
      if (u32_of_lane0(&ds->state) != 1) continue;
      const uint32_t g = u32_of_lane0(&ds->graph), k = u32_of_lane0(&ds->k);
      if (g >= p.ngraphs || k == 0 || k > kServeCols || ((blocked >> g) & 1u)) continue;
      const uint64_t freec = ~(g == 0 ? actv[0] : g == 1 ? actv[1] : g == 2 ? actv[2] : actv[3]);
      if ((uint32_t)__popcll(freec) < k) {
        blocked |= 1u << g;
        continue;
      }
      const bool isfree = (freec >> lane) & 1ull;
      const uint32_t rank = (uint32_t)__popcll(freec & ((1ull << lane) - 1ull));
      const bool take = isfree && rank < k;
      const uint64_t taken = __ballot(take);
      if (take) {
        const uint32_t n = g == 0 ? p.g[0].n : g == 1 ? p.g[1].n : g == 2 ? p.g[2].n : p.g[3].n;
        st->col_out[g][lane] = ds->out + 4ull * rank * n;
        st->col_ticket[g][lane] = t;
        st->col_start[g][lane] = it + 1;  // first expanded by the next iteration's Stage 1
        st->adm_gc[n_admit + rank] = (g << 8) | lane;
        st->adm_src[n_admit + rank] = ds->src[rank];
      }
      n_admit += k;
#pragma unroll
      for (uint32_t h = 0; h < kServeMaxGraphs; ++h)
        if (h == g) actv[h] |= taken;
      if (lane == 0) {
        st->active[g] |= taken;
        st->admitted[g] |= taken;
        st->remaining[r] = k;
        st->maxlev[r] = 0;
        ds->state = 2;
        mb->slot[r].admit_iter = it + 1;
        sys_store(&mb->slot[r].state, 2u);
      }
      __threadfence_block();
      __builtin_amdgcn_wave_barrier();
    }
    // the admitted prefix leaves the window
    while (consumed != seen && u32_of_lane0(&st->slot[consumed % kServeRing].state) >= 2) ++consumed;
    if (lane == 0) st->consumed = consumed;
    uint64_t any_active = 0;
#pragma unroll
    for (uint32_t g = 0; g < kServeMaxGraphs; ++g) any_active |= actv[g];
    if (any_active || n_admit) break;
    // idle: nothing runs and nothing admissible waits
    const uint32_t stop_i = sys_poll(&mb->stop), sub_i = sys_poll(&mb->submitted);
    const uint32_t stop = readlane(stop_i, 0);
    const uint32_t sub2 = readlane(sub_i, 0);
    if (stop == 2 || (stop && consumed == seen && seen == sub2)) {
      exit_now = 1;
      break;
    }
    if (__builtin_amdgcn_s_memrealtime() - t_idle0 > p.idle_limit) {
      exit_now = 1;
      break;
    }
    if (sub2 == seen) __builtin_amdgcn_s_sleep(127);
  }
  if (lane == 0) {
    st->n_admit = n_admit;
    st->exit = exit_now;
    st->iter = it;
  }
}

// ---- admission phase A: clear reused columns, initialise output rows ----
__device__ void serve_init_a(const ServeParams& p) {
  const ServeState* st = p.st;
  const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x, nt = gridDim.x * blockDim.x;
  for (uint32_t g = 0; g < p.ngraphs; ++g) {
    const unsigned long long clr = st->admitted[g] & st->dirty[g];
    if (!clr) continue;
    const ServeGraph& G = p.g[g];
    for (uint32_t u = tid; u < G.n; u += nt) {
      G.vis[2 * (uint64_t)u] &= ~clr;
      G.vis[2 * (uint64_t)u + 1] &= ~clr;
      G.front[u] &= ~clr;
    }
  }
  for (uint32_t i = 0; i < st->n_admit; ++i) {
    const uint32_t g = st->adm_gc[i] >> 8, c = st->adm_gc[i] & 0xFFu;
    const uint32_t n = p.g[g].n;
    int32_t* row = reinterpret_cast<int32_t*>(st->col_out[g][c]);
    for (uint32_t u = tid; u < n; u += nt) row[u] = -1;
  }
}

// ---- admission phase B: source bits, level 0, initial queue entries ----
template <int SIG>
__device__ void serve_init_b(const ServeParams& p, uint32_t it) {
  ServeState* st = p.st;
  const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x, nt = gridDim.x * blockDim.x;
  if (blockIdx.x == 0 && threadIdx.x == 0)
    for (uint32_t g = 0; g < p.ngraphs; ++g) st->dirty[g] &= ~st->admitted[g];
  for (uint32_t i = tid; i < st->n_admit; i += nt) {
    const uint32_t g = st->adm_gc[i] >> 8, c = st->adm_gc[i] & 0xFFu;
    const ServeGraph& G = p.g[g];
    const uint32_t s = st->adm_src[i];
    const unsigned long long bit = 1ull << c;
    atomicOr(G.vis + 2 * (uint64_t)s, bit);
    atomicOr(G.vis + 2 * (uint64_t)s + 1, bit);
    atomicOr(G.front + s, bit);
    G.touched[s] = 2;  // on the frontier
    reinterpret_cast<int32_t*>(st->col_out[g][c])[sorig(G, s)] = 0;
  }
  // the VSS ranges of the sources' slice sets join the next iteration's queue, once per
  // distinct (graph, slice set): one wavefront per admitted column, which appends
  // unless an earlier admitted column names the same set
  const uint32_t wid = tid / kWave, nwv = nt / kWave, lane = lane_id();
  const uint32_t na = st->n_admit;
  for (uint32_t i = wid; i < na; i += nwv) {
    const uint32_t g = st->adm_gc[i] >> 8;
    const uint32_t ss = st->adm_src[i] / SIG;
    bool dup = false;
    for (uint32_t j0 = 0; j0 < i; j0 += kWave) {
      const uint32_t j = j0 + lane;
      dup |= __ballot(j < i && (st->adm_gc[j] >> 8) == g && st->adm_src[j] / SIG == ss) != 0;
    }
    if (dup) continue;
    const ServeGraph& G = p.g[g];
    const uint32_t b = G.real_ptrs[ss], e = G.real_ptrs[ss + 1];
    uint32_t pos = 0;
    if (lane == 0 && e > b) pos = atomicAdd(qlen_of(p, g, it % 3), e - b);
    pos = readlane(pos, 0);
    uint32_t* qc = G.queue + (it & 1) * G.qcap;
    for (uint32_t j = lane; j < e - b; j += kWave) qc[pos + j] = b + j;
  }
}

// ---- Stage 1 over the concatenated queues of every graph ----
template <typename MT, int SLOTS>
__device__ void serve_stage1(const ServeParams& p, uint32_t it, const uint32_t (&len)[kServeMaxGraphs],
                             uint32_t dense) {
  constexpr int SIG = 8 * sizeof(MT);
  uint32_t pre[kServeMaxGraphs + 1];
  pre[0] = 0;
#pragma unroll
  for (uint32_t g = 0; g < kServeMaxGraphs; ++g) pre[g + 1] = pre[g] + (g < p.ngraphs ? len[g] : 0u);
  const uint32_t total = pre[kServeMaxGraphs];
  const uint32_t lane = lane_id();
  const uint32_t wid = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const uint32_t nw = (gridDim.x * blockDim.x) / kWave;
  for (uint32_t base = wid; base < total; base += nw * kWave) {
    const uint32_t pos = base + lane * nw;
    uint32_t mb = 0, me = 0, ms = 0, mg = 0;
    if (pos < total) {
      mg = (pos >= pre[1]) + (pos >= pre[2]) + (pos >= pre[3]);
      const ServeGraph& G = p.g[mg];
      const uint32_t v = (G.queue + ((it - 1) & 1) * G.qcap)[pos - pre[mg]];
      mb = G.vss_beg[v];
      me = G.vss_beg[v + 1];
      ms = G.v2r[v];
    }
    const uint32_t cnt = min((uint32_t)kWave, (total - base + nw - 1) / nw);
    // Two VSSs per step at sigma <= 16 (possibly of different graphs): the B-tile
    // and slice loads of both, then their visited-pair reads, are issued before
    // either is applied, which halves the chain of dependent round trips per VSS.
    // At sigma = 32 two B tiles would not fit the scalar registers.
    constexpr uint32_t P = SIG <= 16 ? 2 : 1;
    for (uint32_t k0 = 0; k0 < cnt; k0 += P) {
      uint32_t gg[P], beg[P], end[P], ss[P];
#pragma unroll
      for (uint32_t h = 0; h < P; ++h) {
        const bool any = k0 + h < cnt;
        const uint32_t k = any ? k0 + h : k0;
        gg[h] = readlane(mg, k);
        beg[h] = readlane(mb, k);
        end[h] = any ? readlane(me, k) : beg[h];  // past the end: an empty VSS
        ss[h] = readlane(ms, k);
      }
      uint64_t bw[P];
#pragma unroll
      for (uint32_t h = 0; h < P; ++h) {
        const ServeGraph& G = p.g[gg[h]];
        const uint32_t col = ss[h] * SIG + lane;
        bw[h] = (lane < (uint32_t)SIG && col < G.n && end[h] > beg[h]) ? G.front[col] : 0ull;
      }
      MT m[P][SLOTS];
      uint32_t u[P][SLOTS];
#pragma unroll
      for (uint32_t h = 0; h < P; ++h) {
        const ServeGraph& G = p.g[gg[h]];
        const MT* masks = static_cast<const MT*>(G.masks);
#pragma unroll
        for (int r = 0; r < SLOTS; ++r) {
          const uint32_t idx = beg[h] + lane + r * kWave;
          const bool ok = idx < end[h];
          m[h][r] = ok ? masks[idx] : MT(0);
          u[h][r] = ok ? G.row_ids[idx] : 0u;
        }
      }
      uint64_t acc[P][SLOTS];
      ulonglong2 cv[P][SLOTS];
#pragma unroll
      for (uint32_t h = 0; h < P; ++h) {
        const ServeGraph& G = p.g[gg[h]];
        uint64_t B[SIG];
#pragma unroll
        for (int j = 0; j < SIG; ++j) B[j] = readlane64(bw[h], j);
#pragma unroll
        for (int r = 0; r < SLOTS; ++r) {
          uint64_t a = 0;
#pragma unroll
          for (int j = 0; j < SIG; ++j) a |= ((uint32_t)m[h][r] >> j & 1u) ? B[j] : 0ull;
          acc[h][r] = a;
          cv[h][r] = reinterpret_cast<const ulonglong2*>(G.vis)[a ? u[h][r] : 0u];
        }
      }
#pragma unroll
      for (uint32_t h = 0; h < P; ++h) {
        const ServeGraph& G = p.g[gg[h]];
        const bool mark = !((dense >> gg[h]) & 1u);
#pragma unroll
        for (int r = 0; r < SLOTS; ++r) {
          const uint64_t fresh = acc[h][r] & ~cv[h][r].x & ~cv[h][r].y;
          if (fresh) {
            atomicOr(G.vis + 2 * (uint64_t)u[h][r] + 1, (unsigned long long)fresh);
            // the first OR that changes u's next word was issued by a thread that read
            // next == current (every iteration starts with them equal)
            if (mark && cv[h][r].y == cv[h][r].x) G.touched[u[h][r]] = 1;
          }
        }
      }
    }
  }
}

// ---- Stage 2 of one graph (as in the k-source kernel, levels per column) ----
template <int SIG>
__device__ void serve_stage2(const ServeParams& p, uint32_t g, uint32_t it, bool dense) {
  constexpr uint32_t L = SIG / 4;  // lanes per slice set
  __shared__ uint32_t s_wave[kMaxWaves];
  __shared__ uint32_t s_base;
  __shared__ uint64_t s_out[kServeCols];
  __shared__ uint32_t s_lvl[kServeCols];
  __shared__ unsigned long long s_grew;
  const ServeGraph& G = p.g[g];
  ServeState* st = p.st;
  const uint32_t lane = lane_id();
  const uint32_t wave = threadIdx.x / kWave, nwaves = blockDim.x / kWave;
  if (threadIdx.x < kServeCols) {
    s_out[threadIdx.x] = st->col_out[g][threadIdx.x];
    s_lvl[threadIdx.x] = it + 1 - st->col_start[g][threadIdx.x];
  }
  if (threadIdx.x == 0) s_grew = 0;
  __syncthreads();
  const uint32_t nq = G.num_sets * L;
  uint32_t* tq = reinterpret_cast<uint32_t*>(G.touched);
  const ulonglong2* vis2 = reinterpret_cast<const ulonglong2*>(G.vis);
  uint32_t* qlen = qlen_of(p, g, it % 3);
  uint32_t* qn = G.queue + (it & 1) * G.qcap;
  uint64_t grew = 0;
  auto write_levels = [&](uint32_t uo, uint64_t diff) {
    uint64_t d = diff;
    while (d) {
      const uint32_t c = __ffsll((unsigned long long)d) - 1;
      reinterpret_cast<int32_t*>(s_out[c])[uo] = (int32_t)s_lvl[c];
      d &= d - 1;
    }
  };
  // Each thread takes kStage2Rounds words per pass (one per grid-sized stride), so
  // that the queue reservation - a block scan, two barriers and an atomic - is paid
  // once per pass instead of once per grid-sized stride: at 4 M vertices and
  // sigma = 8 one pass covers the whole graph.
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t b0 = blockIdx.x * blockDim.x; b0 < nq; b0 += kStage2Rounds * stride) {
    uint32_t cnt = 0, vb[kStage2Rounds], vn[kStage2Rounds];
    uint32_t tw[kStage2Rounds];
    if (!dense) {
      // the state words of every round first, so that their loads overlap
#pragma unroll
      for (uint32_t j = 0; j < kStage2Rounds; ++j) {
        const uint32_t q = b0 + j * stride + threadIdx.x;
        tw[j] = q < nq ? tq[q] : 0u;
      }
    }
#pragma unroll
    for (uint32_t j = 0; j < kStage2Rounds; ++j) {
      const uint32_t q = b0 + j * stride + threadIdx.x;
      const uint32_t base = 4 * (q - lane);
      uint32_t hit = 0;
      if (b0 + j * stride < nq) {  // uniform over the workgroup
        if (dense) {
          // the four vertices' loads first: a store to the visited pairs between
          // them would order each load after the previous vertex's round trip
          ulonglong2 cv[4];
          uint32_t uo[4];
#pragma unroll
          for (uint32_t r = 0; r < 4; ++r) {
            const uint32_t u = base + r * kWave + lane;
            const uint32_t ui = u < G.n ? u : 0u;
            cv[r] = vis2[ui];
            uo[r] = sorig(G, ui);
          }
          uint64_t m[4];
#pragma unroll
          for (uint32_t r = 0; r < 4; ++r) {
            const uint32_t u = base + r * kWave + lane;
            uint64_t diff = 0;
            if (u < G.n) {
              diff = cv[r].y & ~cv[r].x;
              G.front[u] = diff;
              G.touched[u] = diff ? 2 : 0;
              if (diff) {
                G.vis[2 * (uint64_t)u] = cv[r].y;
                write_levels(uo[r], diff);
                grew |= diff;
              }
            }
            m[r] = __ballot(diff != 0);
          }
          const uint32_t r = lane >> 4;
          const uint64_t mr = r == 0 ? m[0] : r == 1 ? m[1] : r == 2 ? m[2] : m[3];
          hit = (uint32_t)(mr >> ((4 * lane) & 63u)) & 0xFu;
        } else {
          hit = tw[j] & 0x01010101u;
          if (__ballot(tw[j] != 0)) {
            // loads of the four vertices first (index 0 for an untouched one), then
            // the stores, so that the round trips overlap
            uint32_t bb[4], uo[4];
            ulonglong2 cv[4];
#pragma unroll
            for (uint32_t r = 0; r < 4; ++r) {
              const uint32_t w = (uint32_t)__shfl((int)tw[j], (int)(r * 16 + (lane >> 2)));
              bb[r] = (w >> (8 * (lane & 3u))) & 0xFFu;
              const uint32_t ui = (bb[r] & 1u) ? base + r * kWave + lane : 0u;
              cv[r] = vis2[ui];
              uo[r] = sorig(G, ui);
            }
#pragma unroll
            for (uint32_t r = 0; r < 4; ++r) {
              const uint32_t u = base + r * kWave + lane;
              if (bb[r] == 2) G.front[u] = 0;
              if (bb[r] & 1u) {
                const uint64_t diff = cv[r].y & ~cv[r].x;
                G.front[u] = diff;
                G.vis[2 * (uint64_t)u] = cv[r].y;
                write_levels(uo[r], diff);
                grew |= diff;
              }
            }
            if (tw[j]) tq[q] = hit << 1;
          }
        }
      }
      const uint64_t act = __ballot(hit != 0);
      constexpr uint64_t kSetLanes = L == 64 ? ~0ull : ((1ull << L) - 1);
      vb[j] = vn[j] = 0;
      if ((lane % L) == 0 && q < nq && ((act >> lane) & kSetLanes)) {
        const uint32_t ss = q / L;
        vb[j] = G.real_ptrs[ss];
        vn[j] = G.real_ptrs[ss + 1] - vb[j];
        cnt += vn[j];
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
    wave_push<kStage2Rounds>(qn, pos, cnt, vb, vn);
    __syncthreads();
  }
  // the columns that grew, ORed within the workgroup first: one device atomic per
  // workgroup instead of one per wavefront on a single word
  grew = wave_or64(grew);
  if (lane == 0 && grew) atomicOr(&s_grew, (unsigned long long)grew);
  __syncthreads();
  if (threadIdx.x == 0 && s_grew) atomicOr(&st->alive[g], s_grew);
  __syncthreads();  // s_out / s_lvl are reloaded for the next graph
}

template <typename MT, int SLOTS>
__global__ __launch_bounds__(1024) void serve_persistent(ServeParams p) {
  constexpr int SIG = 8 * sizeof(MT);
  ServeState* st = p.st;
  uint32_t* ctrl = p.ctrl;
  const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t it = st->iter;  // written by the previous launch (or at creation)
  if (tid == 0) st->launches += 1;
  for (;; ++it) {
    if (tid == 0)
      for (uint32_t g = 0; g < p.ngraphs; ++g)
        __hip_atomic_store(qlen_of(p, g, (it + 1) % 3), 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    uint32_t len[kServeMaxGraphs] = {0, 0, 0, 0};
    uint32_t dense = 0;
    for (uint32_t g = 0; g < p.ngraphs; ++g) {
      len[g] = ld_relaxed(qlen_of(p, g, (it - 1) % 3));
      if ((uint64_t)len[g] * kDenseFrac >= p.g[g].num_vss) dense |= 1u << g;
    }
    // the control wavefront first settles finished and new requests, then joins
    // Stage 1 (whose queue it does not change).  Thread 0, in that wavefront, keeps
    // the phase times.
    const uint64_t t0 = tid == 0 ? __builtin_amdgcn_s_memrealtime() : 0;
    if (blockIdx.x == 0 && threadIdx.x < kWave) serve_control(p, it);
    const uint64_t tc = tid == 0 ? __builtin_amdgcn_s_memrealtime() : 0;
    serve_stage1<MT, SLOTS>(p, it, len, dense);
    grid_barrier(ctrl);
    const uint64_t t1 = tid == 0 ? __builtin_amdgcn_s_memrealtime() : 0;
    if (st->exit) {
      if (tid == 0) {
        st->prof[0] += tc - t0;
        for (int i = 0; i < 5; ++i) p.mb->prof[i] = st->prof[i];
        __threadfence_system();
      }
      break;
    }
    for (uint32_t g = 0; g < p.ngraphs; ++g)
      if (st->active[g]) serve_stage2<SIG>(p, g, it, (dense >> g) & 1u);
    grid_barrier(ctrl);
    const uint64_t t2 = tid == 0 ? __builtin_amdgcn_s_memrealtime() : 0;
    if (st->n_admit) {
      serve_init_a(p);
      grid_barrier(ctrl);
      serve_init_b<SIG>(p, it);
      grid_barrier(ctrl);
    }
    if (tid == 0) {
      const uint64_t t3 = __builtin_amdgcn_s_memrealtime();
      st->prof[0] += tc - t0;
      st->prof[1] += t1 - tc;
      st->prof[2] += t2 - t1;
      st->prof[3] += t3 - t2;
      st->prof[4] += 1;
    }
  }
}

template <typename MT>
const void* ssym(uint32_t slots) {
  switch (slots) {
    case 1: return reinterpret_cast<const void*>(&serve_persistent<MT, 1>);
    case 2: return reinterpret_cast<const void*>(&serve_persistent<MT, 2>);
    case 4: return reinterpret_cast<const void*>(&serve_persistent<MT, 4>);
    case 8: return reinterpret_cast<const void*>(&serve_persistent<MT, 8>);
    default: return nullptr;
  }
}

}  // namespace

const void* serve_kernel_symbol(uint32_t sigma, uint32_t slots) {
  switch (sigma) {
    case 8: return ssym<uint8_t>(slots);
    case 16: return ssym<uint16_t>(slots);
    case 32: return ssym<uint32_t>(slots);
    default: return nullptr;
  }
}

hipError_t launch_serve(const ServeParams& p, uint32_t sigma, uint32_t slots, uint32_t grid, uint32_t block,
                        hipStream_t stream) {
  const void* k = serve_kernel_symbol(sigma, slots);
  if (!k || p.ngraphs == 0 || p.ngraphs > kServeMaxGraphs) return hipErrorInvalidValue;
  ServeParams copy = p;
  void* args[] = {&copy};
  return hipLaunchCooperativeKernel(k, dim3(grid), dim3(block), args, 0, stream);
}

}  // namespace blest
