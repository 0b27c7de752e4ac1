/*
 * blest.h - C-ABI of libblest, a pull-based breadth-first search over Binarised
 * Virtual Slice Sets (BVSS) for AMD Instinct MI355X (gfx950).
 *
 * Method: Elbek and Kaya, "BLEST: Blazingly Efficient BFS using Tensor Cores".
 *   - BFS as repeated Boolean-semiring products y = A (x) x with A the adjacency of
 *     the transposed graph (Section 2).
 *   - Slices, slice sets and virtual slice sets (Sections 2 and 2.1); column-major
 *     placement of a VSS's row-sorted slices (Section 2.1.2).
 *   - Compression-oriented reordering (Algorithm 1, JaccardWithWindows, after a
 *     locality pre-pass where the paper runs Gorder) for social-like graphs and
 *     bandwidth-reducing reordering (RCM) otherwise (Sections 2.2 and 2.2.1).
 *   - The eager kernel (Algorithm 2) and the lazy vertex-update kernel
 *     (Algorithm 3, Section 3.2), all levels fused into one persistent launch
 *     (Section 3.3).
 *   - Multi-source BFS stacks the frontiers column-wise into a frontier matrix
 *     (Section 2); here up to 64 sources share one launch.
 *
 * Conventions common to every call
 *   - Vertices are 0 .. n-1.  The input CSR lists OUT-neighbours; BFS follows
 *     out-edges.  Self-loops and duplicate arcs are accepted and dropped.
 *   - Levels are int32 in the caller's (original) vertex IDs; -1 = unreachable;
 *     the source has level 0.
 *   - Device pointers are plain HIP device addresses; `stream` is a hipStream_t
 *     passed as void* (NULL = the null stream).  BFS calls are asynchronous on
 *     that stream; argument errors are returned synchronously before anything is
 *     enqueued; a launch failure returns BLEST_ERR_DEVICE.
 *   - No C++ exception crosses this interface.  Every call is thread-safe for
 *     distinct handles; calls on one handle from several host threads must be
 *     serialised by the caller.
 */
#ifndef BLEST_H
#define BLEST_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct blest_graph* blest_handle;

typedef enum {
  BLEST_OK = 0,
  BLEST_ERR_INVALID_ARGUMENT = 1, /* null pointer, source >= n, k out of range, ... */
  BLEST_ERR_INVALID_GRAPH = 2,    /* row_ptr not monotone, row_ptr[n] != nnz, col >= n */
  BLEST_ERR_TOO_LARGE = 3,        /* nnz >= 2^32 (the paper's |E| <= 2^32 - 1 limit) */
  BLEST_ERR_OUT_OF_MEMORY = 4,    /* host or device allocation failed */
  BLEST_ERR_BUDGET = 5,           /* a request exceeds the configured device budget */
  BLEST_ERR_DEVICE = 6,           /* a HIP call or kernel launch failed */
  BLEST_ERR_NO_DEVICE = 7,        /* handle built host-only (device = -1) or no GPU */
  BLEST_ERR_INTERNAL = 8
} blest_status;

/* Orderings (Section 2.2).  AUTO applies the paper's static rule (Section 2.2.1):
 * social-like graphs get Algorithm 1, others reverse Cuthill-McKee. */
enum {
  BLEST_REORDER_AUTO = 0,
  BLEST_REORDER_NONE = 1,
  BLEST_REORDER_COMPRESSION = 2, /* Algorithm 1, JaccardWithWindows */
  BLEST_REORDER_BANDWIDTH = 3    /* reverse Cuthill-McKee */
};

/* Vertex-update schemes.  AUTO: lazy (Algorithm 3) iff the graph is social-like
 * and its update divergence exceeds 25,000 (Section 4, discussion of Table 3);
 * otherwise eager (Algorithm 2).  ADAPTIVE chooses per level, on the device, from
 * the level's queue length (the per-level policy the paper leaves to future work,
 * Section 6): levels with fewer than eager_max queued VSSs claim eagerly (one grid
 * barrier, no vertex sweep), others mark lazily and sweep. */
enum { BLEST_UPDATE_AUTO = 0, BLEST_UPDATE_EAGER = 1, BLEST_UPDATE_LAZY = 2, BLEST_UPDATE_ADAPTIVE = 3 };

typedef struct {
  uint32_t sigma;      /* slice width in columns: 8 (the paper's value), 16 or 32 */
  uint32_t slots;      /* slices per lane of a 64-lane wavefront: tau = 64 * slots (1, 2, 4, 8; default 2) */
  uint32_t window;     /* Algorithm 1 window w, a multiple of sigma; 0 = auto (the default): 65536, or
                          4096 after the shingle pre-pass */
  int32_t reorder;     /* BLEST_REORDER_* */
  int32_t update;      /* BLEST_UPDATE_* */
  int32_t device;      /* HIP device ordinal; -1 builds host-only (structure and stats) */
  uint32_t threads;    /* host threads for the build (0 = all hardware threads) */
  uint32_t block;      /* threads per workgroup of the persistent kernels, a multiple of 64 (0 = 1024) */
  uint32_t blocks_per_cu; /* persistent workgroups per compute unit (0 = 1); block * blocks_per_cu <= 2048.
                             The grid is clamped to the workgroups a CU can really hold at once by the
                             kernel's registers and LDS (see blest_stats_t.blocks_per_cu_own) */
  uint32_t group;      /* VSSs whose slice loads a wavefront keeps in flight: 1, 2 or 4 (0 = 2) */
  uint32_t ranges;     /* row ranges of the lazy kernel: a power of two <= 32 (0 = 1).  With R > 1
                          every VSS stays inside one range and workgroup b caches the visited bits
                          of range b % R; one range (the default) caches the lowest rows */
  uint32_t hubs;       /* hub sort after the ordering: sigma-aligned vertex groups reordered by
                          summed in-degree, largest first, groups kept intact (compression is
                          unchanged); 0 = auto (on for social-like graphs), 1 = off, 2 = on */
  uint32_t lds_kib;    /* LDS per workgroup caching visited bits in the lazy Stage 1, in KiB:
                          0 = auto (128, clamped to the device), 1..128, or BLEST_LDS_OFF.  The
                          cache holds the first C words (C a power of two) of every 64-word
                          chunk of the range, C as large as fits */
  uint32_t eager_max;  /* BLEST_UPDATE_ADAPTIVE: levels with fewer queued VSSs run eagerly
                          (0 = num_vss / 32) */
  uint32_t pack;       /* 0 = auto: with sigma 8, slots <= 4 and n <= 2^24 the single-source kernel
                          reads each slice as one 32-bit word (row ID | mask << 24, an extra
                          4 bytes per slice on the device); 1 = off */
  uint32_t multi_ranges; /* k-source kernel: row ranges of its own VSS partition, a power of two
                          <= 32 (0 = 1).  With R > 1 its VSSs are also cut at R row ranges and
                          workgroup b pulls range b % R only, so that each XCD's L2 holds one
                          range's visited pairs */
  uint32_t prepass;    /* locality pre-pass before Algorithm 1 (Section 2.2 runs Gorder there): 0 = auto
                          (on whenever Algorithm 1 runs), 1 = off, 2 = shingle ordering (vertices sorted
                          by min-hashes of their out-neighbour sets, Chierichetti et al., KDD 2009) */
  uint32_t shingles;   /* min-hashes per vertex of the shingle ordering, 1..8 (0 = 2) */
  uint64_t shingle_seed; /* seed of its hash functions: h_i(u) is output u + 1 of the SplitMix64 stream
                          (Steele, Lea and Flood, OOPSLA 2014) seeded with output i + 1 of the stream
                          seeded with shingle_seed (default 0x243F6A8885A308D3) */
  uint32_t max_grid;   /* cap on the workgroups of the single-source persistent launch (0 = every
                          co-resident one).  A smaller grid pays a cheaper grid barrier per level, which
                          suits graphs with thousands of small levels (high diameter) */
} blest_options;

#define BLEST_LDS_OFF 0xFFFFFFFFu

typedef struct {
  uint32_t n;
  uint64_t m;                   /* arcs after dropping loops and duplicates */
  uint32_t sigma, tau, lanes;
  uint32_t num_slice_sets;      /* ceil(n / sigma) */
  uint32_t num_vss;
  uint64_t num_slices;          /* stored = unpadded slices (the layout pads nothing) */
  double compression;           /* m / (num_slices * sigma)            (Section 2.2) */
  double u_div_paper;           /* update divergence, 32 lanes x 32/sigma slots (Section 2.2.1) */
  double u_div_native;          /* same metric on this layout (64 lanes x slots) */
  int32_t social_like;          /* Section 2.2.1 test */
  int32_t reorder_used;         /* BLEST_REORDER_* actually applied */
  int32_t update_used;          /* BLEST_UPDATE_* actually used */
  uint32_t nranges;             /* row ranges of the VSS partition */
  uint32_t range_len;           /* rows per range */
  uint64_t bvss_device_bytes;   /* static arrays resident on the device */
  uint64_t bvss_bytes_table3;   /* the paper's accounting (Table 3) for this structure */
  double reorder_seconds;       /* host ordering time */
  double build_seconds;         /* host BVSS construction time (after ordering) */
  int32_t hubs_sorted;          /* 1 if the hub sort was applied */
  uint32_t lds_bytes;           /* visited bits per workgroup cached in LDS by the lazy kernel */
  uint32_t lds_chunk_words;     /* cached words per 64-word chunk of a range (64 = the whole range) */
  uint32_t hub_cpos;            /* positions per 64-word chunk that the hub sort filled first (0: none) */
  uint32_t grid;                /* workgroups of the single-source persistent launch (0: host-only) */
  uint32_t block;               /* threads per workgroup of the persistent launches */
  uint32_t kernel_vgprs;        /* vector registers per lane of the single-source kernel */
  uint32_t blocks_per_cu_runtime; /* workgroups per CU the runtime's occupancy query allows */
  uint32_t blocks_per_cu_own;   /* workgroups per CU by the kernel's registers and LDS (gfx950 rules);
                                   the grid uses the smaller of the two and blocks_per_cu */
  uint32_t eager_max;           /* adaptive threshold in effect (queued VSSs) */
  int32_t packed;               /* 1 if the single-source kernel reads packed slices */
  uint32_t multi_ranges;        /* row ranges of the k-source kernel's VSS partition */
  uint32_t multi_num_vss;       /* VSSs of that partition */
  int32_t prepass_used;         /* 1 if the shingle pre-pass ran before Algorithm 1 */
  double prepass_seconds;       /* its host time (included in reorder_seconds) */
  uint32_t window_used;         /* Algorithm 1 window applied (0: Algorithm 1 did not run) */
} blest_stats_t;

/* Fills *opt with the defaults listed above. */
void blest_default_options(blest_options* opt);

/* Builds the reordered BVSS of G = (V, E) and, unless opt->device == -1, uploads
 * it to that device.  row_ptr (n + 1 entries) and col_idx (nnz entries) are HOST
 * arrays holding the out-neighbour CSR; they are copied, so the caller may free
 * them on return.  opt may be NULL (defaults).  On success *out owns all device
 * memory of the graph; release it with blest_destroy.  Errors: INVALID_ARGUMENT
 * (null pointers, n == 0, bad option values), INVALID_GRAPH, TOO_LARGE,
 * OUT_OF_MEMORY, DEVICE. */
blest_status blest_build(uint32_t n, uint64_t nnz, const uint32_t* row_ptr, const uint32_t* col_idx,
                         const blest_options* opt, blest_handle* out);

/* Single-source BFS (Algorithm 2 or 3, per the handle's update scheme).
 * levels_out: DEVICE int32[n], caller-owned, fully overwritten.
 * parents_out: DEVICE int32[n] or NULL; if given, parents_out[v] is the smallest
 * original ID among v's in-neighbours one level closer to the source, the source's
 * parent is itself, and -1 marks unreached vertices.
 * Errors: INVALID_ARGUMENT (source >= n, null levels_out), NO_DEVICE, DEVICE. */
blest_status blest_bfs(blest_handle h, uint32_t source, int32_t* levels_out, int32_t* parents_out,
                       void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): blest_bfs without the
 * parents output, whose per-call state (visited bits, reached bytes, frontier
 * bitmaps, queues, control block) lives in a static device array of
 * BLEST_NOALLOC_SCRATCH_BYTES that the library holds on every device it runs on
 * until the process ends, instead of the per-stream workspace that blest_bfs
 * allocates on a stream's first call.  The call allocates nothing (no hipMalloc,
 * hipFree or event creation) and needs n/8 + n + 3n/8 bytes plus 12, 16 or 24 bytes
 * per VSS of queues (eager, lazy, adaptive scheme), each part rounded up to 256,
 * plus a 2 KiB control block; a graph needing more
 * returns BLEST_ERR_BUDGET before anything is enqueued.  Every call on a device
 * shares that device's scratch, which keeps the last call's contents; the call
 * clears what must start at zero.  The library orders every persistent launch on
 * a device behind the previous one, so calls from several streams do not run at
 * once; work that bypassed that order and used the same scratch would race.
 * Arguments, levels_out and errors as for blest_bfs. */
#define BLEST_NOALLOC_SCRATCH_BYTES (64u << 20)
blest_status blest_bfs_noalloc(blest_handle h, uint32_t source, int32_t* levels_out, void* stream);

/* k-source BFS in one launch: sources is a HOST array of k vertex IDs
 * (1 <= k <= 64, repeats allowed); levels_out is DEVICE int32[k * n], row j
 * (levels_out[j*n .. j*n+n-1]) belongs to sources[j].  The frontiers form an
 * n x k bit-matrix (Section 2); each level is one Boolean SpMM over the BVSS.
 * Errors: INVALID_ARGUMENT, NO_DEVICE, DEVICE. */
blest_status blest_bfs_multi(blest_handle h, const uint32_t* sources, uint32_t k, int32_t* levels_out,
                             void* stream);

/* One launch running g independent single-source BFSs, BFS i on graph hs[i] from
 * sources[i] (a HOST array), writing DEVICE int32[n_i] at levels_out[i] (a HOST
 * array of g device pointers).  All handles must live on the same device and share
 * sigma and slots.  Each BFS is owned by one workgroup whose bitmaps live in LDS,
 * so graphs must have n <= 131072; larger ones return INVALID_ARGUMENT.  The item
 * table is uploaded synchronously; the launch itself is asynchronous on `stream`
 * and the table is released once a later call sees the launch finished.  This is
 * blest_batch_create + blest_batch_run in one call. */
blest_status blest_bfs_many(const blest_handle* hs, const uint32_t* sources, uint32_t g,
                            int32_t* const* levels_out, void* stream);

/* A reusable many-graphs launch: the item table (arguments as for blest_bfs_many)
 * is built and uploaded once; blest_batch_run enqueues the single ordinary
 * (non-cooperative) launch and nothing else, so it can be captured into a HIP
 * graph and replayed.  The handles and output buffers must outlive the batch.
 * blest_batch_destroy must not be called while a run is in flight. */
typedef struct blest_batch* blest_batch_handle;
blest_status blest_batch_create(const blest_handle* hs, const uint32_t* sources, uint32_t g,
                                int32_t* const* levels_out, blest_batch_handle* out);
blest_status blest_batch_run(blest_batch_handle b, void* stream);
void blest_batch_destroy(blest_batch_handle b);

/* Continuous batching (a request loop against resident graphs).  A server owns
 * one persistent launch on its own stream that serves BFS requests of 1..64
 * sources on up to 4 resident graphs (handles built on one device with the same
 * sigma and slots).  Every graph has 64 source columns; at every level boundary
 * the launch admits waiting requests, oldest first per graph, into free columns,
 * so a request that arrives while others run joins the running sweep instead of
 * waiting for it, and its rows advance one level per server iteration like the
 * others'.  A request's rows are the k-source BFS of its sources (Section 2's
 * stacked frontiers): identical to blest_bfs_multi of the same sources alone.
 * Requests are exchanged through a ring of 256 slots in pinned host memory; the
 * launch ends by itself after idle_ms (0 = 20) milliseconds without work and is
 * started again by the next submit or poll.  Device memory: the server holds
 * 24 n + n + 16 num_vss bytes per graph for the column state; the caller
 * provides each request's output and the server admits a request only while the
 * outputs of submitted, unreleased requests stay within budget_bytes.  Graph
 * handles must outlive the server; other persistent launches on the device wait
 * while a server launch runs.
 * Errors: INVALID_ARGUMENT (count 0 or > 4, null handles, mixed devices, sigma or
 * slots), NO_DEVICE, TOO_LARGE, OUT_OF_MEMORY, DEVICE. */
typedef struct blest_server* blest_server_handle;
blest_status blest_server_create(const blest_handle* graphs, uint32_t count, uint64_t budget_bytes, uint32_t idle_ms,
                                 blest_server_handle* out);

/* Submits k sources (HOST array, original IDs) on graphs[graph]; levels_out is
 * DEVICE int32[k * n], row j for sources[j], fully written by the server before
 * the request reports done.  *ticket identifies the request.  Returns
 * BLEST_ERR_BUDGET, with nothing submitted, when the request's 4 k n output bytes
 * would take the unreleased outputs past budget_bytes or when the oldest ring
 * slot is still held by an unreleased request: release finished requests and
 * submit again.  Errors: INVALID_ARGUMENT, BUDGET, DEVICE. */
blest_status blest_server_submit(blest_server_handle s, uint32_t graph, const uint32_t* sources, uint32_t k,
                                 int32_t* levels_out, uint64_t* ticket);

/* Non-blocking state of a request: *state = 0 waiting, 1 running, 2 done (its
 * levels are complete in device memory); levels = 1 + its deepest level; the
 * server iterations that admitted it and after which it finished (either pointer
 * may be NULL).  Starts a new launch if the request waits and none runs.
 * Errors: INVALID_ARGUMENT (unknown or released ticket), DEVICE. */
blest_status blest_server_poll(blest_server_handle s, uint64_t ticket, int32_t* state, uint32_t* levels,
                               uint32_t* admit_iter, uint32_t* done_iter);

/* Releases a done request: its ring slot and its output bytes return to the
 * budget (the output buffer stays the caller's).  Errors: INVALID_ARGUMENT (not
 * done, unknown or already released). */
blest_status blest_server_release(blest_server_handle s, uint64_t ticket);

typedef struct {
  uint64_t budget;            /* output bytes the server may have outstanding */
  uint64_t outstanding;       /* output bytes of submitted, unreleased requests */
  uint64_t peak_outstanding;  /* largest value `outstanding` reached */
  uint64_t resident_bytes;    /* device memory held by the server itself */
  uint64_t submitted;         /* requests submitted so far */
  uint64_t launches;          /* persistent launches started so far */
  int32_t running;            /* a launch is in flight */
  uint32_t grid, block;       /* launch shape */
  /* device-side phase times, totals over the launches that have ended (read them
   * once `running` is 0): server iterations, and microseconds spent in the
   * control step, in Stage 1 up to its grid barrier (the control step runs beside
   * the other workgroups' Stage 1), in Stage 2 up to its barrier, and in
   * admissions */
  uint64_t iterations;
  double control_us, stage1_us, stage2_us, admit_us;
} blest_server_stats_t;
blest_status blest_server_stats(blest_server_handle s, blest_server_stats_t* out);

/* Asks the launch to end once nothing waits or runs and waits for that at most
 * timeout_ms (0 = 60000) milliseconds; past that it tells the launch to end at
 * its next level boundary, running requests or not (they never report done), and
 * waits as long again.  Then frees the server.  If the launch still runs, returns
 * BLEST_ERR_DEVICE and frees nothing (the call may be repeated).  NULL is
 * ignored. */
blest_status blest_server_destroy(blest_server_handle s, uint32_t timeout_ms);

/* Changes the launch settings of a built handle without rebuilding it: update
 * scheme (BLEST_UPDATE_*), threads per workgroup, workgroups per compute unit, VSS
 * group depth and the adaptive scheme's eager_max, with the meanings (and 0 =
 * default) of blest_options.  Used by autotuning.  Must not be called while work
 * on the handle is in flight.
 * Errors: INVALID_ARGUMENT (bad values; the handle is left unchanged), DEVICE. */
blest_status blest_configure(blest_handle h, int32_t update, uint32_t block, uint32_t blocks_per_cu, uint32_t group,
                             uint32_t eager_max);

/* Structure statistics of a built handle (host-side, no device access). */
blest_status blest_stats(blest_handle h, blest_stats_t* out);

/* Device bytes a k-source call on this handle needs beyond the resident BVSS
 * (frontier/visited bitmaps, queues, and k * n * 4 bytes of levels), for
 * admission control.  k = 0 reports the resident BVSS bytes alone. */
blest_status blest_footprint(blest_handle h, uint32_t k, uint64_t* device_bytes);

/* Host copies of internal arrays, for structural tests and accounting.
 * which: BLEST_EXPORT_*; dst may be NULL to query *size_bytes; otherwise at most
 * capacity_bytes are copied. */
enum {
  BLEST_EXPORT_NEW_ID = 0,          /* uint32[n]: new label of each original vertex */
  BLEST_EXPORT_REAL_PTRS = 1,       /* uint32[num_slice_sets + 1] */
  BLEST_EXPORT_VIRTUAL_TO_REAL = 2, /* uint32[num_vss] */
  BLEST_EXPORT_VSS_BEGIN = 3,       /* uint32[num_vss + 1]: first slice of each VSS */
  BLEST_EXPORT_ROW_IDS = 4,         /* uint32[num_slices], new labels */
  BLEST_EXPORT_MASKS = 5,           /* sigma/8 bytes per slice, little-endian, bit j = column j */
  BLEST_EXPORT_VSS_RANGE = 6,       /* uint8[num_vss]: row range of each VSS */
  BLEST_EXPORT_ORDER_ID = 7,        /* uint32[n]: label of each original vertex after the ordering
                                       alone (pre-pass and Algorithm 1, or RCM), before the hub sort */
  BLEST_EXPORT_PREPASS_ID = 8       /* uint32[n]: label of each original vertex after the shingle
                                       pre-pass alone (the identity when it did not run) */
};
blest_status blest_export(blest_handle h, int32_t which, void* dst, uint64_t capacity_bytes,
                          uint64_t* size_bytes);

/* Per-source statistics of a DEVICE level array (k rows of n int32, row j the
 * levels from source j, -1 = unreached; the layout blest_bfs_multi writes), for
 * the multi-source analytics the stacked frontiers of Section 2 serve (centrality,
 * diameter).  Writes to DEVICE arrays of k entries: reached[j] = number of
 * levels >= 0, total[j] = their sum, ecc[j] = their maximum (-1 for an empty
 * row), far[j] = the smallest vertex at level ecc[j] (0xFFFFFFFF for an empty
 * row) and closeness[j] = (reached[j] - 1) / total[j] in double precision (0 when
 * total[j] = 0).  Runs on `stream` (hipStream_t, NULL = default) of `device`
 * without host synchronisation and allocates nothing; the outputs must not alias
 * `levels`.  k = 0 does nothing.  Errors: INVALID_ARGUMENT (k > 65535 or a null
 * pointer), NO_DEVICE, DEVICE (launch failure). */
blest_status blest_level_stats(int32_t device, const int32_t* levels, uint32_t k, uint32_t n, uint64_t* reached,
                               uint64_t* total, int32_t* ecc, uint32_t* far, double* closeness, void* stream);

/* Algorithmic device bytes of one BFS call whose result is `levels` (HOST int32,
 * k rows of n in original IDs, k = 1 for blest_bfs, 1..64 for blest_bfs_multi):
 * for every iteration l and every slice set holding a vertex of level l - 1 in any
 * row, its unpadded slices (4-byte row ID + sigma/8-byte mask), its frontier (the
 * sigma-bit chunk, or sigma 64-bit words when k > 1) and 8 bytes per VSS (queue
 * entry + VSS metadata); plus, for k = 1, the lazy scheme's per-level sweep of the
 * two n-bit visited bitmaps, the 4n-byte level initialisation and 4 bytes per
 * reached vertex (its level write) (the sweep counted for the iterations the
 * handle's scheme runs lazily: all, none, or, adaptive, those whose queue holds
 * at least eager_max VSSs); for k > 1, per
 * iteration, a 25n-byte vertex sweep when the queue holds at least 1/16 of the
 * VSSs, else n state bytes plus 26 bytes per vertex changed in the iteration and 8
 * per vertex leaving the frontier; the 4kn-byte initialisation and 4 bytes per
 * reached (source, vertex) pair.  Lets a benchmark turn a measured time into GB/s.
 * Errors: INVALID_ARGUMENT. */
blest_status blest_model_bytes(blest_handle h, const int32_t* levels, uint32_t k, uint64_t* bytes);

/* Measures the grid barrier of the persistent launches (one workgroup of `block`
 * threads per compute unit, at most max_grid workgroups when max_grid > 0, as
 * blest_options.max_grid caps them): a launch doing `rounds` barriers and nothing
 * else, timed with HIP events after a warm-up run; *seconds_per_barrier = time /
 * rounds.  For the latency bound of high-diameter graphs, where every level costs
 * at least one barrier.  Synchronous; allocates a small control block.
 * Errors: INVALID_ARGUMENT, NO_DEVICE, DEVICE. */
blest_status blest_barrier_probe(int32_t device, uint32_t block, uint32_t max_grid, uint32_t rounds,
                                 double* seconds_per_barrier);

/* Releases the library's process-wide HIP objects once the work using them has
 * finished: the per-device events that order persistent launches and the item
 * tables of finished blest_bfs_many launches.  For an orderly exit while the HIP
 * runtime is still up (the Python binding calls it at interpreter exit).  Handles
 * built before the call can afterwards only be destroyed; handles built after it
 * work normally. */
void blest_shutdown(void);

/* Releases the handle and its device memory.  NULL is ignored.  Must not be called
 * while work using the handle is still pending on a stream. */
void blest_destroy(blest_handle h);

/* Static string naming a status code. */
const char* blest_status_string(blest_status s);

#ifdef __cplusplus
}
#endif

#endif /* BLEST_H */
