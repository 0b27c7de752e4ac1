// Device-side entry points of libblest (defined in kernels.hip), called by capi.cpp.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace blest {

// Control block shared by the persistent kernels (uint32 words).  Each counter
// sits on its own 128-byte line.
constexpr uint32_t kLine = 32;                       // uint32 per 128-byte line
constexpr uint32_t kBarGroups = 8;                   // one arrival counter per XCD
constexpr uint32_t kBarRoot = kBarGroups * kLine;    // root arrival counter
constexpr uint32_t kBarGen = kBarRoot + kLine;       // generation word
constexpr uint32_t kQlen = kBarGen + kLine;          // 4 queue-length counters
constexpr uint32_t kCtrlWords = kQlen + 4 * kLine;

struct BfsParams {
  // static BVSS (read-only during a launch)
  const uint32_t* row_ids;
  const void* masks;
  const uint32_t* vss_beg;
  const uint32_t* v2r;
  const uint32_t* real_ptrs;
  const uint32_t* orig_id;  // new label -> original ID, 32 * n_words entries; nullptr = identity
  const uint8_t* vss_range; // row range of each VSS
  const uint32_t* packed;   // sigma = 8: row ID | mask << 24 per slice (nullptr: separate arrays)
  // per-call workspace
  uint32_t* vis;            // visited bits, n_words
  uint8_t* mark;            // lazy: reached byte per vertex, 32 * n_words
  uint32_t* front;          // eager, adaptive: 3 * n_words (the lazy scheme keeps alpha in its queue entries)
  uint32_t* queue;          // eager: 3 * qcap 32-bit entries; lazy: 2, adaptive: 3 * qcap 64-bit entries (VSS, alpha)
  uint32_t* ctrl;           // kCtrlWords
  int32_t* levels;          // n, original IDs
  uint32_t n, n_words, num_sets, num_vss, qcap;
  uint32_t src;             // source, new label
  uint32_t nranges;         // row ranges (a power of two, at most kMaxRanges)
  uint32_t range_len;       // rows per range (a multiple of 32)
  uint32_t range_words;     // visited words of a range cached in LDS (0: none)
  uint32_t lds_cshift;      // the cache holds words 0 .. 2^lds_cshift - 1 of every 64-word chunk
  uint32_t lds_min_len;     // lazy: levels with fewer queue entries skip the LDS cache
  uint32_t eager_max;       // adaptive: levels with fewer queued VSSs claim eagerly
};

// Queue entries carry the VSS's row range in their low bits.
constexpr uint32_t kRangeBits = 5;
constexpr uint32_t kMaxRanges = 1u << kRangeBits;
constexpr uint32_t kMaxLdsBytes = 128 * 1024;

// Persistent single-source BFS.  mode: 0 = Algorithm 2 (eager) every level,
// 1 = Algorithm 3 (lazy) every level, 2 = per level by queue length (adaptive).
// grid must be co-resident (the call uses a cooperative launch) and a multiple of
// p.nranges.  group = VSSs whose slice loads a wavefront keeps in flight together
// (1, 2, 4).  With p.range_words > 0 the lazy kernel caches, per workgroup, the
// visited words 0 .. 2^lds_cshift - 1 of every 64-word chunk of the workgroup's
// row range in LDS (4 * range_words bytes of dynamic LDS); other rows are checked
// in memory.
hipError_t launch_bfs(const BfsParams& p, uint32_t sigma, uint32_t slots, int mode, uint32_t group, uint32_t grid,
                      uint32_t block, hipStream_t stream);

// Returns the kernel symbol used by launch_bfs (for occupancy queries).
const void* bfs_kernel_symbol(uint32_t sigma, uint32_t slots, int mode, uint32_t group, bool lds, bool packed);

// k-source BFS (k <= 64): per-vertex 64-bit frontier and visited words, bit j for
// source j.
constexpr uint32_t kMaxSources = 64;
struct MultiParams {
  const uint32_t* row_ids;
  const void* masks;
  const uint32_t* vss_beg;
  const uint32_t* v2r;
  const uint32_t* real_ptrs;
  const uint32_t* orig_id;        // nullptr = identity
  unsigned long long* vis;        // 2 * n: (current, next) per vertex
  unsigned long long* front;      // n
  uint8_t* touched;               // num_sets * sigma bytes: vertex got new bits this level
  uint32_t* queue;                // 2 * qcap
  uint32_t* ctrl;                 // kCtrlWords
  int32_t* levels;                // k * n, original IDs, row j for source j
  const uint8_t* vss_range;        // row range of each VSS (nullptr when nranges == 1)
  uint32_t nranges;                // row ranges of this kernel's VSS partition (grid is a multiple)
  uint32_t n, num_sets, num_vss, qcap, k, n_init_sets;
  uint32_t src[kMaxSources];       // new labels
  uint32_t init_sets[kMaxSources]; // distinct slice sets holding a source
};

hipError_t launch_bfs_multi(const MultiParams& p, uint32_t sigma, uint32_t slots, uint32_t grid, uint32_t block,
                            hipStream_t stream);
const void* bfs_multi_kernel_symbol(uint32_t sigma, uint32_t slots);

// ---- continuous-batching server (kernels_serve.hip) ----
// One persistent launch serves BFS requests of 1..64 sources on up to
// kServeMaxGraphs resident graphs.  Every graph has 64 source columns (one bit of
// a 64-bit word per vertex, as in the k-source kernel); a request takes k free
// columns of its graph at a level boundary and frees them when its last column
// stops growing, so requests that arrive while others run join the running
// sweeps instead of waiting for them.
constexpr uint32_t kServeMaxGraphs = 4;
constexpr uint32_t kServeCols = 64;
constexpr uint32_t kServeRing = 256;  // request slots of the mailbox ring

// Request slot (host memory, coherent).  The host fills a free slot and then
// publishes it by advancing ServeMailbox::submitted; afterwards only the device
// writes the slot (state, admit_iter, done_iter, levels) until the host sees
// state 3 and frees it.
struct ServeSlot {
  uint32_t state;       // 0 free, 1 submitted, 2 admitted, 3 done
  uint32_t graph;       // index of the resident graph
  uint32_t k;           // sources (1..64)
  uint32_t admit_iter;  // server iteration whose level boundary admitted the request
  uint32_t done_iter;   // iteration after which its last column stopped growing
  uint32_t levels;      // 1 + largest level over its rows
  uint64_t out;         // device int32[k * n], row j for src[j], original IDs
  uint32_t src[kServeCols];  // sources, new labels
};

struct ServeMailbox {
  uint32_t submitted;  // tickets [0, submitted) are published (host writes)
  uint32_t stop;       // host: 1 = end the launch once no request is waiting or running
  uint32_t pad0[2];
  // totals over all launches so far, written when a launch ends: realtime ticks
  // (100 MHz) spent in the control step, in Stage 1 up to its grid barrier, in
  // Stage 2 up to its barrier and in admissions, and the iteration count
  uint64_t prof[5];
  uint32_t pad[18];
  ServeSlot slot[kServeRing];
};

struct ServeGraph {
  const uint32_t* row_ids;
  const void* masks;
  const uint32_t* vss_beg;
  const uint32_t* v2r;
  const uint32_t* real_ptrs;
  const uint32_t* orig_id;    // nullptr = identity
  unsigned long long* vis;    // 2 * n: (current, next) per vertex
  unsigned long long* front;  // n
  uint8_t* touched;           // num_sets * sigma state bytes
  uint32_t* queue;            // 2 * qcap
  uint32_t n, num_sets, num_vss, qcap;
};

// Device-resident server state; persists across launches (zeroed at creation).
struct ServeState {
  uint32_t consumed;   // tickets below this are admitted or done
  uint32_t seen;       // tickets below this are copied into `slot`
  uint32_t iter;       // server iterations so far (monotone across launches)
  uint32_t exit;       // set by the control step: the launch ends
  uint32_t n_admit;    // columns admitted at this level boundary
  uint32_t launches;   // launches that started
  uint32_t pad0[2];
  uint64_t prof[5];    // running totals of ServeMailbox::prof
  unsigned long long active[kServeMaxGraphs];  // columns in use
  unsigned long long alive[kServeMaxGraphs];   // columns that grew in the last iteration
  unsigned long long dirty[kServeMaxGraphs];   // freed columns whose bits are still set
  unsigned long long admitted[kServeMaxGraphs];  // columns admitted at this boundary
  uint64_t col_out[kServeMaxGraphs][kServeCols];   // row pointer of each column
  uint32_t col_ticket[kServeMaxGraphs][kServeCols];
  uint32_t col_start[kServeMaxGraphs][kServeCols];  // iteration of admission
  uint32_t remaining[kServeRing];                   // running columns per slot
  uint32_t maxlev[kServeRing];
  ServeSlot slot[kServeRing];                       // device copies of published slots
  uint32_t adm_gc[kServeMaxGraphs * kServeCols];    // (graph << 8) | column
  uint32_t adm_src[kServeMaxGraphs * kServeCols];   // source (new label)
};

struct ServeParams {
  ServeGraph g[kServeMaxGraphs];
  uint32_t ngraphs;
  uint32_t idle_limit;   // realtime ticks (100 MHz) without work before the launch ends
  ServeMailbox* mb;      // host memory, coherent
  ServeState* st;        // device memory
  uint32_t* ctrl;        // barrier counters and queue lengths (kServeCtrlWords)
};
constexpr uint32_t kServeCtrlWords = kQlen + 3 * kServeMaxGraphs * kLine;

hipError_t launch_serve(const ServeParams& p, uint32_t sigma, uint32_t slots, uint32_t grid, uint32_t block,
                        hipStream_t stream);
const void* serve_kernel_symbol(uint32_t sigma, uint32_t slots);

// Many independent single-source BFSs in one ordinary launch: workgroup i runs
// item i start to finish, with its bitmaps in LDS and only workgroup barriers.
struct ManyItem {
  const uint32_t* row_ids;
  const void* masks;
  const uint32_t* vss_beg;
  const uint32_t* v2r;
  const uint32_t* real_ptrs;
  const uint32_t* orig_id;  // nullptr = identity
  int32_t* levels;          // n, original IDs
  uint32_t* queue;          // 2 * max(num_vss, 1)
  uint32_t n, num_vss, src, pad;
};
constexpr uint32_t kManyMaxN = 131072;  // LDS holds 3 bits per vertex
constexpr uint32_t kManyBlock = 512;

// items: device array of g descriptors; all items share sigma and slots.
hipError_t launch_bfs_many(const ManyItem* items, uint32_t g, uint32_t max_n, uint32_t sigma, uint32_t slots,
                           hipStream_t stream);

// Parents post-pass: parent[v] = smallest original ID among the in-neighbours of v
// on level level[v] - 1.  Ordinary launches on `stream`.
// Per-row reached count, level sum, eccentricity, smallest farthest vertex and
// closeness of a k x n level array (k <= 65535).
hipError_t launch_level_stats(const int32_t* levels, uint32_t k, uint32_t n, unsigned long long* reached,
                              unsigned long long* total, int32_t* ecc, uint32_t* far, double* closeness,
                              uint32_t num_cus, hipStream_t stream);
hipError_t launch_parents(const BfsParams& p, uint32_t sigma, const int32_t* levels, int32_t* parents,
                          hipStream_t stream);

// Device address of the allocation-free entry point's static scratch array on
// `device` (which must be the current device); looked up once per device.
hipError_t noalloc_scratch(int device, void** ptr);

// A persistent launch doing `rounds` grid barriers (ctrl: kCtrlWords, zeroed).
hipError_t launch_barrier_probe(uint32_t* ctrl, uint32_t rounds, uint32_t grid, uint32_t block, hipStream_t stream);
const void* barrier_probe_symbol();

// Zeroes n 32-bit words at p with one small ordinary launch on `stream`.
hipError_t launch_zero_words(uint32_t* p, uint32_t n, hipStream_t stream);

}  // namespace blest
