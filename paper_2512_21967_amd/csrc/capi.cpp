// The C-ABI of libblest (include/blest.h): argument checking, host-side build,
// device residency, per-stream workspaces and kernel launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstddef>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "../../include/blest.h"
#include "internal.hpp"
#include "kernels.hpp"

using namespace blest;

namespace {

// Device buffer that frees itself.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  hipError_t alloc(size_t b) {
    bytes = b;
    return hipMalloc(&p, b ? b : 4);
  }
  template <class T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

// Per-stream scratch of the single-source kernels.  Calls on one stream are
// ordered, so reusing the stream's workspace is safe without host waits.
struct SingleWorkspace {
  DevBuf vis, mark, front, queue, ctrl;
};

// Per-stream scratch of the k-source kernel: 64-bit visited pairs and frontier
// words per vertex, two queues, control block.
struct MultiWorkspace {
  DevBuf vis, front, touched, queue, ctrl;
};

// Persistent launches are serialised device-wide: two persistent grids that each
// wait for all of their workgroups could otherwise starve one another of compute
// units.  Every persistent launch waits on the previous one's completion event.
struct DeviceSerial {
  std::mutex mu;
  hipEvent_t last = nullptr;
};
DeviceSerial g_serial[64];

// Lazy levels with fewer queued VSSs than min(kLdsMinQueue, cached words / 16)
// check visited bits in memory only: refilling the LDS cache costs about as much
// as such a level's checks.
constexpr uint32_t kLdsMinQueue = 4096;
// Default Algorithm 1 windows.  After the shingle pre-pass, vertices with shared
// neighbours are already close, and a small window keeps nearly all of the
// compression (R-MAT scale 22: 0.1400 at 4096 against 0.1416 at 65536) at a
// fraction of the ordering time, which grows with the window once the candidate
// lists of a window are dense.
constexpr uint32_t kWindowAlone = 1u << 16;
constexpr uint32_t kWindowAfterPrepass = 1u << 12;

}  // namespace

struct blest_batch;
struct blest_server;

struct blest_graph {
  blest_options opt{};
  uint32_t n = 0;
  uint64_t m = 0;
  Bvss bvss;
  std::vector<uint32_t> new_id;   // original -> new
  std::vector<uint32_t> order_id; // original -> label after the ordering alone (before the hub sort)
  std::vector<uint32_t> prepass_id; // original -> label after the shingle pre-pass alone (empty: none)
  int prepass_used = 0;
  uint32_t window_used = 0;  // Algorithm 1 window (0: Algorithm 1 did not run)
  double prepass_seconds = 0;
  std::vector<uint32_t> orig_id;  // new -> original
  bool identity = true;
  int mode = 0;  // kernel scheme: 0 eager (Algorithm 2), 1 lazy (Algorithm 3), 2 adaptive per level
  int social = 0;
  int hubs_sorted = 0;
  int reorder_used = BLEST_REORDER_NONE;
  double u_div_paper = 0, u_div_native = 0, compression = 0;
  double reorder_seconds = 0, build_seconds = 0;
  // device state
  bool on_device = false;
  int device = -1;
  DevBuf d_row_ids, d_masks, d_vss_beg, d_v2r, d_real_ptrs, d_orig_id, d_vss_range, d_packed;
  bool packed = false;  // the single-source kernel reads slices packed (sigma 8, row IDs < 2^24)
  // The k-source kernel's own VSS partition, cut at multi_ranges row ranges (used
  // when multi_ranges > 1; the slices are shared with the base partition).
  uint32_t multi_ranges = 1;
  VssPartition mpart;
  DevBuf d_m_real_ptrs, d_m_v2r, d_m_vss_beg, d_m_vss_range;
  uint32_t nranges = 1, range_len = 0, range_words = 0;
  uint32_t lds_cap_words = 0, lds_cshift = 0, hub_cpos = 0;
  uint32_t grid = 0, block = 0;
  uint32_t occ_api = 0, occ_own = 0;  // workgroups per CU: runtime answer, own resource bound
  int num_regs = 0;                   // vector registers of the single-source kernel
  std::mutex ws_mu;
  std::map<void*, std::unique_ptr<SingleWorkspace>> single_ws;
  std::map<void*, std::unique_ptr<MultiWorkspace>> multi_ws;
  uint32_t multi_grid = 0;
  uint32_t n_words() const { return (n + 31) / 32; }
  uint32_t orig_id_of(uint32_t u) const { return identity ? u : orig_id[u]; }
};

// A device-resident table of (graph, source, output) items for the many-graphs
// launch.  Items are sorted by stored slices, largest first.
struct blest_batch {
  int device = -1;
  uint32_t g = 0, max_n = 0, sigma = 8, slots = 4;
  DevBuf d_items, d_queues;
};

// A continuous-batching server over resident graphs (kernels_serve.hip).
struct blest_server {
  int device = -1;
  uint32_t sigma = 8, slots = 2, grid = 0, block = 1024;
  std::vector<blest_graph*> graphs;
  struct GraphState {
    DevBuf vis, front, touched, queue;
  };
  std::vector<std::unique_ptr<GraphState>> gs;
  DevBuf state, ctrl;
  ServeMailbox* mb = nullptr;      // pinned host memory, coherent
  ServeMailbox* mb_dev = nullptr;  // its device address
  hipStream_t stream = nullptr;
  hipEvent_t ev = nullptr;         // recorded after every launch
  bool launched = false;
  uint64_t budget = 0, outstanding = 0, peak = 0, resident = 0;
  uint32_t next_ticket = 0, idle_limit = 0;
  uint64_t launches = 0;
  uint64_t charge[kServeRing] = {};
  std::mutex mu;
  ~blest_server() {
    if (ev) (void)hipEventDestroy(ev);
    if (stream) (void)hipStreamDestroy(stream);
    if (mb) (void)hipHostFree(mb);
  }
};

namespace {

// Completed-launch bookkeeping for blest_bfs_many's internal batches.
struct PendingBatch {
  blest_batch* b;
  hipEvent_t done;
};
std::mutex g_pending_mu;
std::vector<PendingBatch> g_pending;

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

blest_status map_rc(int rc) {
  switch (rc) {
    case kOk: return BLEST_OK;
    case kInvalidGraph: return BLEST_ERR_INVALID_GRAPH;
    case kTooLarge: return BLEST_ERR_TOO_LARGE;
    case kNoMemory: return BLEST_ERR_OUT_OF_MEMORY;
    default: return BLEST_ERR_INTERNAL;
  }
}

bool valid_options(const blest_options& o) {
  if (o.sigma != 8 && o.sigma != 16 && o.sigma != 32) return false;
  if (o.slots != 1 && o.slots != 2 && o.slots != 4 && o.slots != 8) return false;
  if (o.window % o.sigma != 0) return false;  // 0 = auto
  if (o.reorder < BLEST_REORDER_AUTO || o.reorder > BLEST_REORDER_BANDWIDTH) return false;
  if (o.update < BLEST_UPDATE_AUTO || o.update > BLEST_UPDATE_ADAPTIVE) return false;
  if (o.block % 64 != 0 || o.block > 1024) return false;
  if (o.blocks_per_cu > 16) return false;
  // at most a compute unit's 2048 threads; the grid is further clamped to what the
  // kernel's registers and LDS let the CU hold at once (own_blocks_per_cu)
  if ((uint64_t)o.block * (o.blocks_per_cu ? o.blocks_per_cu : 1) > 2048) return false;
  if (o.group != 1 && o.group != 2 && o.group != 4) return false;
  if (o.ranges > kMaxRanges || (o.ranges & (o.ranges - 1)) != 0) return false;
  if (o.hubs > 2) return false;
  if (o.lds_kib != BLEST_LDS_OFF && o.lds_kib > kMaxLdsBytes / 1024) return false;
  if (o.pack > 1) return false;
  if (o.multi_ranges > kMaxRanges || (o.multi_ranges & (o.multi_ranges - 1)) != 0) return false;
  if (o.prepass > 2 || o.shingles > 8) return false;
  return true;
}

template <class T>
hipError_t upload(DevBuf& d, const std::vector<T>& h) {
  hipError_t e = d.alloc(sizeof(T) * std::max<size_t>(h.size(), 1));
  if (e != hipSuccess) return e;
  if (h.empty()) return hipSuccess;
  return hipMemcpy(d.p, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice);
}

blest_status set_grid(blest_graph* g);
hipError_t serial_event(int device);

// Kernel scheme of an update option.  AUTO is the paper's static rule: lazy iff
// the graph is social-like and its update divergence exceeds 25,000 (Section 4,
// discussion of Table 3).
int mode_of(int32_t update, int social, double u_div) {
  switch (update) {
    case BLEST_UPDATE_EAGER: return 0;
    case BLEST_UPDATE_LAZY: return 1;
    case BLEST_UPDATE_ADAPTIVE: return 2;
    default: return social && u_div > 25000.0 ? 1 : 0;
  }
}

// Adaptive scheme: levels whose queue holds fewer VSSs than this claim eagerly.
// Default 1/32 of the VSSs: on R-MAT scale 22 the first two and last two levels
// (1 to 23,741 VSSs) run eagerly, the three dense ones (136K to 1.07M) lazily; on a
// mesh every level (a few hundred VSSs) runs eagerly.
uint32_t eager_max_of(const blest_graph* g);

blest_status to_device(blest_graph* g) {
  if (hipSetDevice(g->device) != hipSuccess) return BLEST_ERR_NO_DEVICE;
  const Bvss& b = g->bvss;
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = upload(g->d_row_ids, b.row_ids);
  if (e == hipSuccess) e = upload(g->d_masks, b.masks);
  if (e == hipSuccess) e = upload(g->d_vss_beg, b.vss_beg);
  if (e == hipSuccess) e = upload(g->d_v2r, b.v2r);
  if (e == hipSuccess) e = upload(g->d_real_ptrs, b.real_ptrs);
  if (e == hipSuccess && !g->identity) {
    // padded to whole 32-vertex words: the lazy kernel loads a word's IDs as vectors
    std::vector<uint32_t> padded(g->orig_id);
    padded.resize(32ull * g->n_words(), 0u);
    e = upload(g->d_orig_id, padded);
  }
  if (e == hipSuccess) e = upload(g->d_vss_range, b.vss_range);
  if (e == hipSuccess && g->multi_ranges > 1) e = upload(g->d_m_real_ptrs, g->mpart.real_ptrs);
  if (e == hipSuccess && g->multi_ranges > 1) e = upload(g->d_m_v2r, g->mpart.v2r);
  if (e == hipSuccess && g->multi_ranges > 1) e = upload(g->d_m_vss_beg, g->mpart.vss_beg);
  if (e == hipSuccess && g->multi_ranges > 1) e = upload(g->d_m_vss_range, g->mpart.vss_range);
  // packed slices for the single-source kernel: row ID | mask << 24
  g->packed = g->opt.pack == 0 && b.sigma == 8 && b.slots <= 4 && g->n <= (1u << 24);
  if (e == hipSuccess && g->packed) {
    std::vector<uint32_t> pk(b.num_slices);
    for (uint64_t k = 0; k < b.num_slices; ++k) pk[k] = b.row_ids[k] | ((uint32_t)b.masks[k] << 24);
    e = upload(g->d_packed, pk);
  }
  if (e == hipErrorOutOfMemory) return BLEST_ERR_OUT_OF_MEMORY;
  if (e != hipSuccess) return BLEST_ERR_DEVICE;
  blest_status st = set_grid(g);
  if (st != BLEST_OK) return st;
  if (serial_event(g->device) != hipSuccess) return BLEST_ERR_DEVICE;
  g->on_device = true;
  return BLEST_OK;
}

// Workgroups of `block` threads that one compute unit can hold at once by the
// kernel's own register, scratch and LDS use, under gfx950's rules: each SIMD
// has 512 vector registers per lane (architectural and accumulation registers
// together), allocated in granules of 8, and 800 scalar registers allocated in
// granules of 16, and runs at most 8 wavefronts; a workgroup's wavefronts are
// spread evenly over the CU's 4 SIMDs; a CU has 160 KiB of LDS.  The runtime
// reports no scalar-register count, and every persistent kernel of this library
// allocates 98-106 of them, which caps it at 7 wavefronts per SIMD: two
// 1024-thread workgroups (8 per SIMD) never fit one CU, whatever the vector
// registers allow.  The runtime's occupancy answer is not taken alone: a
// persistent grid larger than what is really resident never gets past its
// first grid barrier.  Kernels with a private segment (scratch) are held to one
// workgroup per CU, since scratch wavefronts are limited per queue as well.
uint32_t own_blocks_per_cu(const void* kernel, uint32_t block, uint32_t dyn_lds, int* num_regs) {
  hipFuncAttributes fa{};
  if (hipFuncGetAttributes(&fa, kernel) != hipSuccess) return 0;
  *num_regs = fa.numRegs;
  constexpr uint32_t kRegsPerLane = 512, kGranule = 8, kMaxWavesPerSimd = 7, kSimds = 4;
  constexpr uint64_t kLdsPerCu = 160ull * 1024;
  const uint32_t regs = std::max<uint32_t>(kGranule, ((uint32_t)std::max(fa.numRegs, 1) + kGranule - 1) / kGranule * kGranule);
  const uint32_t waves_per_simd = std::min(kMaxWavesPerSimd, kRegsPerLane / regs);
  const uint32_t waves = (block + 63) / 64;
  const uint32_t per_simd = (waves + kSimds - 1) / kSimds;  // a workgroup's wavefronts on each SIMD
  uint32_t nb = per_simd ? waves_per_simd / per_simd : 0;
  const uint64_t lds = (uint64_t)fa.sharedSizeBytes + dyn_lds;
  if (lds) nb = std::min<uint64_t>(nb, kLdsPerCu / lds);
  if (fa.localSizeBytes > 0) nb = std::min<uint32_t>(nb, 1);
  return nb;
}

uint32_t eager_max_of(const blest_graph* g) {
  if (g->opt.eager_max) return g->opt.eager_max;
  return std::max<uint32_t>(1, g->bvss.num_vss / 32);
}

// Persistent grid: co-resident workgroups, capped at blocks_per_cu per CU.
blest_status set_grid(blest_graph* g) {
  const Bvss& b = g->bvss;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, g->device) != hipSuccess || cus <= 0)
    return BLEST_ERR_DEVICE;
  g->block = g->opt.block;
  const bool lds = g->mode != 0 && g->range_words > 0;
  const void* k = bfs_kernel_symbol(b.sigma, b.slots, g->mode, g->opt.group, lds, g->packed);
  if (lds) {
    // the LDS cache takes what the device leaves beside the kernel's static LDS
    int max_lds = 0;
    hipFuncAttributes fa{};
    if (hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, g->device) != hipSuccess ||
        hipFuncGetAttributes(&fa, k) != hipSuccess)
      return BLEST_ERR_DEVICE;
    const int64_t room = ((int64_t)max_lds - (int64_t)fa.sharedSizeBytes) / 4;
    if (room < 1) return BLEST_ERR_DEVICE;
    g->range_words = cache_shape(g->range_len / 32, std::min<uint32_t>(g->lds_cap_words, (uint32_t)room),
                                 g->lds_cshift);
    if (g->range_words == 0) return BLEST_ERR_DEVICE;
    // the attribute belongs to the kernel, not to this graph: it is set to all the
    // room there is, so that a graph with a smaller cache built later does not
    // shrink it below what this one launches with
    if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)(4 * room)) != hipSuccess)
      return BLEST_ERR_DEVICE;
  }
  const uint32_t dyn = lds ? 4 * g->range_words : 0;
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, (int)g->block, dyn) != hipSuccess || nb <= 0)
    return BLEST_ERR_DEVICE;
  g->occ_api = (uint32_t)nb;
  g->occ_own = own_blocks_per_cu(k, g->block, dyn, &g->num_regs);
  const uint32_t per_cu = std::min({(uint32_t)nb, g->occ_own, g->opt.blocks_per_cu});
  g->grid = per_cu * (uint32_t)cus / g->nranges * g->nranges;
  if (g->opt.max_grid && g->grid > g->opt.max_grid)
    g->grid = std::max(g->nranges, g->opt.max_grid / g->nranges * g->nranges);
  if (g->grid == 0) return BLEST_ERR_DEVICE;
  const void* km = bfs_multi_kernel_symbol(b.sigma, b.slots);
  int nbm = 0, regs_m = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nbm, km, (int)g->block, 0) != hipSuccess || nbm <= 0)
    return BLEST_ERR_DEVICE;
  const uint32_t own_m = own_blocks_per_cu(km, g->block, 0, &regs_m);
  g->multi_grid = std::min({(uint32_t)nbm, own_m, g->opt.blocks_per_cu}) * (uint32_t)cus / g->multi_ranges *
                  g->multi_ranges;
  if (g->multi_grid == 0) return BLEST_ERR_DEVICE;
  return BLEST_OK;
}

SingleWorkspace* single_workspace(blest_graph* g, void* stream, blest_status* st) {
  std::lock_guard<std::mutex> lk(g->ws_mu);
  auto it = g->single_ws.find(stream);
  if (it != g->single_ws.end()) return it->second.get();
  auto ws = std::make_unique<SingleWorkspace>();
  const size_t nw = g->n_words();
  hipError_t e = ws->vis.alloc(sizeof(uint32_t) * nw);
  if (e == hipSuccess) e = ws->mark.alloc(32 * nw);
  if (e == hipSuccess) e = ws->front.alloc(sizeof(uint32_t) * 3 * nw);
  // queues: eager 3 x 32-bit entries, lazy 2 and adaptive 3 x 64-bit entries (VSS, alpha)
  if (e == hipSuccess) e = ws->queue.alloc(sizeof(uint32_t) * 6 * std::max<size_t>(g->bvss.num_vss, 1));
  if (e == hipSuccess) e = ws->ctrl.alloc(sizeof(uint32_t) * kCtrlWords);
  if (e == hipSuccess) e = hipMemset(ws->ctrl.p, 0, sizeof(uint32_t) * kCtrlWords);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    *st = e == hipErrorOutOfMemory ? BLEST_ERR_OUT_OF_MEMORY : BLEST_ERR_DEVICE;
    return nullptr;
  }
  SingleWorkspace* raw = ws.get();
  g->single_ws.emplace(stream, std::move(ws));
  return raw;
}

MultiWorkspace* multi_workspace(blest_graph* g, void* stream, blest_status* st) {
  std::lock_guard<std::mutex> lk(g->ws_mu);
  auto it = g->multi_ws.find(stream);
  if (it != g->multi_ws.end()) return it->second.get();
  auto ws = std::make_unique<MultiWorkspace>();
  const size_t n = g->n;
  hipError_t e = ws->vis.alloc(16 * n);
  if (e == hipSuccess) e = ws->front.alloc(8 * n);
  if (e == hipSuccess) e = ws->touched.alloc((size_t)std::max<uint32_t>(g->bvss.num_sets, 1) * g->bvss.sigma);
  const size_t qv = std::max<size_t>(g->multi_ranges > 1 ? g->mpart.num_vss : g->bvss.num_vss, 1);
  if (e == hipSuccess) e = ws->queue.alloc(sizeof(uint32_t) * 2 * qv);
  if (e == hipSuccess) e = ws->ctrl.alloc(sizeof(uint32_t) * kCtrlWords);
  if (e == hipSuccess) e = hipMemset(ws->ctrl.p, 0, sizeof(uint32_t) * kCtrlWords);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    *st = e == hipErrorOutOfMemory ? BLEST_ERR_OUT_OF_MEMORY : BLEST_ERR_DEVICE;
    return nullptr;
  }
  MultiWorkspace* raw = ws.get();
  g->multi_ws.emplace(stream, std::move(ws));
  return raw;
}

// Creates the device's tail event (at upload time, so that launches create nothing).
hipError_t serial_event(int device) {
  DeviceSerial& ds = g_serial[device & 63];
  std::lock_guard<std::mutex> lk(ds.mu);
  if (ds.last) return hipSuccess;
  return hipEventCreateWithFlags(&ds.last, hipEventDisableTiming);
}

// Makes `stream` wait for the previous persistent launch on this device, runs
// `launch`, and records the new tail event.
template <class F>
hipError_t serial_launch(int device, hipStream_t stream, F&& launch) {
  DeviceSerial& ds = g_serial[device & 63];
  std::lock_guard<std::mutex> lk(ds.mu);
  if (!ds.last) return hipErrorNotReady;  // created when a handle is uploaded (serial_event)
  hipError_t e = hipStreamWaitEvent(stream, ds.last, 0);
  if (e != hipSuccess) return e;
  e = launch();
  if (e != hipSuccess) return e;
  return hipEventRecord(ds.last, stream);
}

BfsParams base_params(const blest_graph* g) {
  BfsParams p{};
  p.row_ids = g->d_row_ids.as<uint32_t>();
  p.masks = g->d_masks.p;
  p.vss_beg = g->d_vss_beg.as<uint32_t>();
  p.v2r = g->d_v2r.as<uint32_t>();
  p.real_ptrs = g->d_real_ptrs.as<uint32_t>();
  p.orig_id = g->identity ? nullptr : g->d_orig_id.as<uint32_t>();
  p.n = g->n;
  p.n_words = g->n_words();
  p.num_sets = g->bvss.num_sets;
  p.num_vss = g->bvss.num_vss;
  p.qcap = std::max<uint32_t>(g->bvss.num_vss, 1);
  p.vss_range = g->d_vss_range.as<uint8_t>();
  p.packed = g->packed ? g->d_packed.as<uint32_t>() : nullptr;
  p.nranges = g->nranges;
  p.range_len = g->range_len;
  p.range_words = g->mode != 0 ? g->range_words : 0;
  p.eager_max = eager_max_of(g);
  p.lds_cshift = g->lds_cshift;
  p.lds_min_len = std::min<uint32_t>(kLdsMinQueue, std::max<uint32_t>(1, p.range_words / 16));
  return p;
}

// Starts a server launch unless one is running.  Caller holds sv->mu.
hipError_t server_ensure_running(blest_server* sv) {
  if (sv->launched && hipEventQuery(sv->ev) == hipErrorNotReady) return hipSuccess;
  ServeParams p{};
  p.ngraphs = (uint32_t)sv->graphs.size();
  for (uint32_t i = 0; i < p.ngraphs; ++i) {
    const blest_graph* h = sv->graphs[i];
    ServeGraph& G = p.g[i];
    G.row_ids = h->d_row_ids.as<uint32_t>();
    G.masks = h->d_masks.p;
    G.vss_beg = h->d_vss_beg.as<uint32_t>();
    G.v2r = h->d_v2r.as<uint32_t>();
    G.real_ptrs = h->d_real_ptrs.as<uint32_t>();
    G.orig_id = h->identity ? nullptr : h->d_orig_id.as<uint32_t>();
    G.vis = sv->gs[i]->vis.as<unsigned long long>();
    G.front = sv->gs[i]->front.as<unsigned long long>();
    G.touched = sv->gs[i]->touched.as<uint8_t>();
    G.queue = sv->gs[i]->queue.as<uint32_t>();
    G.n = h->n;
    G.num_sets = h->bvss.num_sets;
    G.num_vss = h->bvss.num_vss;
    G.qcap = 2 * std::max<uint32_t>(h->bvss.num_vss, 1);
  }
  p.idle_limit = sv->idle_limit;
  p.mb = sv->mb_dev;
  p.st = sv->state.as<ServeState>();
  p.ctrl = sv->ctrl.as<uint32_t>();
  if (hipSetDevice(sv->device) != hipSuccess) return hipErrorInvalidDevice;
  hipError_t e = serial_launch(sv->device, sv->stream, [&] {
    return launch_serve(p, sv->sigma, sv->slots, sv->grid, sv->block, sv->stream);
  });
  if (e == hipSuccess) e = hipEventRecord(sv->ev, sv->stream);
  if (e == hipSuccess) {
    sv->launched = true;
    ++sv->launches;
  }
  return e;
}

}  // namespace

extern "C" {

void blest_default_options(blest_options* o) {
  if (!o) return;
  o->sigma = 8;
  o->slots = 2;
  o->window = 0;
  o->reorder = BLEST_REORDER_AUTO;
  o->update = BLEST_UPDATE_AUTO;
  o->device = 0;
  o->threads = 0;
  o->block = 1024;
  o->blocks_per_cu = 1;
  o->group = 2;
  o->ranges = 0;
  o->hubs = 0;
  o->lds_kib = 0;
  o->eager_max = 0;
  o->pack = 0;
  o->multi_ranges = 0;
  o->prepass = 0;
  o->shingles = 0;
  o->shingle_seed = 0x243F6A8885A308D3ull;
  o->max_grid = 0;
}

blest_status blest_build(uint32_t n, uint64_t nnz, const uint32_t* row_ptr, const uint32_t* col_idx,
                         const blest_options* opt, blest_handle* out) {
  if (!out) return BLEST_ERR_INVALID_ARGUMENT;
  *out = nullptr;
  if (n == 0 || !row_ptr || (nnz > 0 && !col_idx)) return BLEST_ERR_INVALID_ARGUMENT;
  if (nnz > 0xFFFFFFFFull) return BLEST_ERR_TOO_LARGE;
  // reached bytes are addressed with 32-bit offsets
  if (32ull * ((n + 31ull) / 32) > 0xFFFFFFFFull) return BLEST_ERR_TOO_LARGE;
  blest_options o;
  blest_default_options(&o);
  if (opt) o = *opt;
  if (o.block == 0) o.block = 1024;
  if (o.blocks_per_cu == 0) o.blocks_per_cu = 1;
  if (o.group == 0) o.group = 2;
  if (!valid_options(o)) return BLEST_ERR_INVALID_ARGUMENT;
  std::unique_ptr<blest_graph> g;
  try {
    g = std::make_unique<blest_graph>();
    g->opt = o;
    g->n = n;
    const int T = (int)o.threads;
    Csr csr;
    int rc = normalise(n, nnz, row_ptr, col_idx, T, csr);
    if (rc != kOk) return map_rc(rc);
    g->m = csr.nnz();
    double t0 = now_s();
    g->social = social_like(csr) ? 1 : 0;
    int reorder = o.reorder;
    if (reorder == BLEST_REORDER_AUTO) reorder = g->social ? BLEST_REORDER_COMPRESSION : BLEST_REORDER_BANDWIDTH;
    g->reorder_used = reorder;
    Csr work;
    if (reorder == BLEST_REORDER_NONE) {
      work = std::move(csr);
    } else {
      Csr gt;
      transpose(csr, gt);
      const bool prepass = reorder == BLEST_REORDER_COMPRESSION && o.prepass != 1;
      if (reorder == BLEST_REORDER_COMPRESSION)
        g->window_used = o.window ? o.window : prepass ? kWindowAfterPrepass : kWindowAlone;
      if (prepass) {
        // shingle pre-pass, then Algorithm 1's windows over the pre-pass labels
        const double tp = now_s();
        shingle_order(csr, o.shingles ? o.shingles : 2, o.shingle_seed, T, g->prepass_id);
        Csr pre, pret;
        relabel(csr, g->prepass_id, T, pre);
        transpose(pre, pret);
        g->prepass_used = 1;
        g->prepass_seconds = now_s() - tp;
        std::vector<uint32_t> win_id;
        jaccard_windows(pre, pret, o.sigma, g->window_used, T, win_id);
        g->new_id.resize(n);
        for (uint32_t v = 0; v < n; ++v) g->new_id[v] = win_id[g->prepass_id[v]];
      } else if (reorder == BLEST_REORDER_COMPRESSION) {
        jaccard_windows(csr, gt, o.sigma, g->window_used, T, g->new_id);
      } else {
        Csr und;
        undirected(csr, gt, und);
        rcm(und, g->new_id);
      }
      relabel(csr, g->new_id, T, work);
      g->identity = false;
      g->orig_id.assign(n, 0);
      for (uint32_t v = 0; v < n; ++v) g->orig_id[g->new_id[v]] = v;
    }
    if (g->identity) {
      g->new_id.resize(n);
      for (uint32_t v = 0; v < n; ++v) g->new_id[v] = v;
    }
    double t1 = now_s();
    g->reorder_seconds = t1 - t0;
    rc = build_slices(work, o.sigma, o.slots, T, g->bvss);
    if (rc != kOk) return map_rc(rc);
    g->compression = g->bvss.num_slices ? (double)g->m / ((double)g->bvss.num_slices * o.sigma) : 0.0;
    // the update-scheme policy reads the divergence of the ordering itself
    g->u_div_paper = update_divergence(g->bvss, 32, 32 / o.sigma);
    g->mode = mode_of(o.update, g->social, g->u_div_paper);
    // Row ranges: with R > 1 every VSS is cut at range boundaries and workgroup b
    // caches range b % R.  The cut multiplies the VSS count (3.6x at R-MAT scale 22
    // with R = 8) and each frontier vertex is then marked by up to R workgroups,
    // which costs more than the global visited checks it saves, so the default is
    // one range, of which the LDS cache holds the first C words of every 64-word
    // chunk (all of it when it fits).
    const uint32_t nw = (n + 31) / 32;
    const uint32_t R = o.ranges ? o.ranges : 1;
    const uint32_t rw = (nw + R - 1) / R;  // visited words per range
    g->nranges = R;
    g->range_len = rw * 32;
    g->lds_cap_words = o.lds_kib == BLEST_LDS_OFF ? 0u : (o.lds_kib ? o.lds_kib * 1024u : kMaxLdsBytes) / 4;
    g->range_words = cache_shape(rw, g->lds_cap_words, g->lds_cshift);
    g->order_id = g->new_id;
    if (o.hubs == 2 || (o.hubs == 0 && g->social)) {
      // Hub sort: the rows that most visited checks land on move into the cached
      // positions (one range) or to the lowest IDs (several ranges).
      g->hub_cpos = R == 1 && g->range_words ? 1u << g->lds_cshift : 0u;
      std::vector<uint32_t> hub_id;
      hub_sort(work, o.sigma, g->hub_cpos, hub_id);
      Csr sorted;
      relabel(work, hub_id, T, sorted);
      work = std::move(sorted);
      for (uint32_t v = 0; v < n; ++v) g->new_id[v] = hub_id[g->new_id[v]];
      g->identity = false;
      g->orig_id.assign(n, 0);
      for (uint32_t v = 0; v < n; ++v) g->orig_id[g->new_id[v]] = v;
      g->hubs_sorted = 1;
      rc = build_slices(work, o.sigma, o.slots, T, g->bvss);
      if (rc != kOk) return map_rc(rc);
    }
    rc = partition_vss(g->bvss, R > 1 ? g->range_len : 0, T);
    if (rc != kOk) return map_rc(rc);
    if (g->bvss.num_vss >= (1u << (32 - kRangeBits))) return BLEST_ERR_TOO_LARGE;
    g->multi_ranges = o.multi_ranges ? o.multi_ranges : 1;
    if (g->multi_ranges > 1) {
      const uint32_t rwm = (nw + g->multi_ranges - 1) / g->multi_ranges;
      partition_vss_into(g->bvss, rwm * 32, T, g->mpart);
      if (g->mpart.num_vss >= (1u << (32 - kRangeBits))) return BLEST_ERR_TOO_LARGE;
    }
    g->build_seconds = now_s() - t1;
    g->u_div_native = update_divergence(g->bvss, 64, 0);
    if (o.device >= 0) {
      g->device = o.device;
      blest_status st = to_device(g.get());
      if (st != BLEST_OK) return st;
    }
  } catch (const std::bad_alloc&) {
    return BLEST_ERR_OUT_OF_MEMORY;
  } catch (...) {
    return BLEST_ERR_INTERNAL;
  }
  *out = g.release();
  return BLEST_OK;
}

blest_status blest_bfs(blest_handle h, uint32_t source, int32_t* levels_out, int32_t* parents_out,
                       void* stream) {
  if (!h || !levels_out) return BLEST_ERR_INVALID_ARGUMENT;
  if (source >= h->n) return BLEST_ERR_INVALID_ARGUMENT;
  if (!h->on_device) return BLEST_ERR_NO_DEVICE;
  try {
    if (hipSetDevice(h->device) != hipSuccess) return BLEST_ERR_DEVICE;
    blest_status st = BLEST_OK;
    SingleWorkspace* ws = single_workspace(h, stream, &st);
    if (!ws) return st;
    BfsParams p = base_params(h);
    p.vis = ws->vis.as<uint32_t>();
    p.mark = ws->mark.as<uint8_t>();
    p.front = ws->front.as<uint32_t>();
    p.queue = ws->queue.as<uint32_t>();
    p.ctrl = ws->ctrl.as<uint32_t>();
    p.levels = levels_out;
    p.src = h->new_id[source];
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = serial_launch(h->device, s, [&] {
      return launch_bfs(p, h->bvss.sigma, h->bvss.slots, h->mode, h->opt.group, h->grid, h->block, s);
    });
    if (e == hipSuccess && parents_out) e = launch_parents(p, h->bvss.sigma, levels_out, parents_out, s);
    return e == hipSuccess ? BLEST_OK : BLEST_ERR_DEVICE;
  } catch (...) {
    return BLEST_ERR_INTERNAL;
  }
}

blest_status blest_bfs_noalloc(blest_handle h, uint32_t source, int32_t* levels_out, void* stream) {
  if (!h || !levels_out) return BLEST_ERR_INVALID_ARGUMENT;
  if (source >= h->n) return BLEST_ERR_INVALID_ARGUMENT;
  // the per-call state, carved out of the static scratch in 256-byte-aligned parts
  const uint64_t nw = h->n_words();
  // queues: eager 3 x 4 bytes, lazy 2 x 8 and adaptive 3 x 8 bytes per VSS
  const uint64_t qbytes = h->mode == 0 ? 12 : h->mode == 1 ? 16 : 24;
  const uint64_t parts[5] = {4 * nw, 32 * nw, 12 * nw, qbytes * std::max<uint32_t>(h->bvss.num_vss, 1),
                             4ull * kCtrlWords};
  uint64_t off[5], need = 0;
  for (int i = 0; i < 5; ++i) {
    off[i] = need;
    need += (parts[i] + 255) / 256 * 256;
  }
  if (need > BLEST_NOALLOC_SCRATCH_BYTES) return BLEST_ERR_BUDGET;
  if (!h->on_device) return BLEST_ERR_NO_DEVICE;
  try {
    if (hipSetDevice(h->device) != hipSuccess) return BLEST_ERR_DEVICE;
    void* base = nullptr;
    if (noalloc_scratch(h->device, &base) != hipSuccess || !base) return BLEST_ERR_DEVICE;
    char* sb = static_cast<char*>(base);
    BfsParams p = base_params(h);
    p.vis = reinterpret_cast<uint32_t*>(sb + off[0]);
    p.mark = reinterpret_cast<uint8_t*>(sb + off[1]);
    p.front = reinterpret_cast<uint32_t*>(sb + off[2]);
    p.queue = reinterpret_cast<uint32_t*>(sb + off[3]);
    p.ctrl = reinterpret_cast<uint32_t*>(sb + off[4]);
    p.levels = levels_out;
    p.src = h->new_id[source];
    hipStream_t s = static_cast<hipStream_t>(stream);
    // The scratch keeps the last call's contents: the barrier counters and queue
    // lengths are cleared by a fill kernel, ordered with the BFS launch behind the
    // previous persistent launch on the device.
    hipError_t e = serial_launch(h->device, s, [&] {
      hipError_t z = launch_zero_words(p.ctrl, kCtrlWords, s);
      if (z != hipSuccess) return z;
      return launch_bfs(p, h->bvss.sigma, h->bvss.slots, h->mode, h->opt.group, h->grid, h->block, s);
    });
    return e == hipSuccess ? BLEST_OK : BLEST_ERR_DEVICE;
  } catch (...) {
    return BLEST_ERR_INTERNAL;
  }
}

blest_status blest_bfs_multi(blest_handle h, const uint32_t* sources, uint32_t k, int32_t* levels_out,
                             void* stream) {
  if (!h || !sources || !levels_out || k == 0 || k > 64) return BLEST_ERR_INVALID_ARGUMENT;
  for (uint32_t j = 0; j < k; ++j)
    if (sources[j] >= h->n) return BLEST_ERR_INVALID_ARGUMENT;
  if (!h->on_device) return BLEST_ERR_NO_DEVICE;
  try {
    if (hipSetDevice(h->device) != hipSuccess) return BLEST_ERR_DEVICE;
    blest_status st = BLEST_OK;
    MultiWorkspace* ws = multi_workspace(h, stream, &st);
    if (!ws) return st;
    MultiParams p{};
    const bool mr = h->multi_ranges > 1;
    p.row_ids = h->d_row_ids.as<uint32_t>();
    p.masks = h->d_masks.p;
    p.vss_beg = (mr ? h->d_m_vss_beg : h->d_vss_beg).as<uint32_t>();
    p.v2r = (mr ? h->d_m_v2r : h->d_v2r).as<uint32_t>();
    p.real_ptrs = (mr ? h->d_m_real_ptrs : h->d_real_ptrs).as<uint32_t>();
    p.vss_range = mr ? h->d_m_vss_range.as<uint8_t>() : nullptr;
    p.nranges = h->multi_ranges;
    p.orig_id = h->identity ? nullptr : h->d_orig_id.as<uint32_t>();
    p.vis = ws->vis.as<unsigned long long>();
    p.front = ws->front.as<unsigned long long>();
    p.touched = ws->touched.as<uint8_t>();
    p.queue = ws->queue.as<uint32_t>();
    p.ctrl = ws->ctrl.as<uint32_t>();
    p.levels = levels_out;
    p.n = h->n;
    p.num_sets = h->bvss.num_sets;
    p.num_vss = mr ? h->mpart.num_vss : h->bvss.num_vss;
    p.qcap = std::max<uint32_t>(p.num_vss, 1);
    p.k = k;
    for (uint32_t j = 0; j < k; ++j) {
      p.src[j] = h->new_id[sources[j]];
      const uint32_t ss = p.src[j] / h->bvss.sigma;
      bool seen = false;
      for (uint32_t i = 0; i < p.n_init_sets; ++i) seen |= p.init_sets[i] == ss;
      if (!seen) p.init_sets[p.n_init_sets++] = ss;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = serial_launch(h->device, s, [&] {
      return launch_bfs_multi(p, h->bvss.sigma, h->bvss.slots, h->multi_grid, h->block, s);
    });
    return e == hipSuccess ? BLEST_OK : BLEST_ERR_DEVICE;
  } catch (...) {
    return BLEST_ERR_INTERNAL;
  }
}

blest_status blest_batch_create(const blest_handle* hs, const uint32_t* sources, uint32_t g,
                                int32_t* const* levels_out, blest_batch_handle* out) {
  if (!out) return BLEST_ERR_INVALID_ARGUMENT;
  *out = nullptr;
  if (!hs || !sources || !levels_out || g == 0) return BLEST_ERR_INVALID_ARGUMENT;
  for (uint32_t i = 0; i < g; ++i) {
    if (!hs[i] || !levels_out[i] || sources[i] >= hs[i]->n) return BLEST_ERR_INVALID_ARGUMENT;
    if (hs[i]->n > kManyMaxN) return BLEST_ERR_INVALID_ARGUMENT;
    if (hs[i]->bvss.sigma != hs[0]->bvss.sigma || hs[i]->bvss.slots != hs[0]->bvss.slots)
      return BLEST_ERR_INVALID_ARGUMENT;
  }
  for (uint32_t i = 0; i < g; ++i) {
    if (!hs[i]->on_device) return BLEST_ERR_NO_DEVICE;
    if (hs[i]->device != hs[0]->device) return BLEST_ERR_INVALID_ARGUMENT;
  }
  try {
    if (hipSetDevice(hs[0]->device) != hipSuccess) return BLEST_ERR_DEVICE;
    std::unique_ptr<blest_batch> b(new blest_batch);
    b->device = hs[0]->device;
    b->g = g;
    b->sigma = hs[0]->bvss.sigma;
    b->slots = hs[0]->bvss.slots;
    std::vector<uint32_t> order(g);
    for (uint32_t i = 0; i < g; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t c) {
      return hs[a]->bvss.num_slices > hs[c]->bvss.num_slices;
    });
    uint64_t qwords = 0;
    for (uint32_t i = 0; i < g; ++i) {
      qwords += 2ull * std::max<uint32_t>(hs[i]->bvss.num_vss, 1);
      b->max_n = std::max(b->max_n, hs[i]->n);
    }
    hipError_t e = b->d_queues.alloc(4 * qwords);
    if (e == hipSuccess) e = b->d_items.alloc(sizeof(ManyItem) * g);
    if (e != hipSuccess) return e == hipErrorOutOfMemory ? BLEST_ERR_OUT_OF_MEMORY : BLEST_ERR_DEVICE;
    std::vector<ManyItem> items(g);
    uint64_t qoff = 0;
    for (uint32_t r = 0; r < g; ++r) {
      const blest_graph* h = hs[order[r]];
      ManyItem& it = items[r];
      it.row_ids = h->d_row_ids.as<uint32_t>();
      it.masks = h->d_masks.p;
      it.vss_beg = h->d_vss_beg.as<uint32_t>();
      it.v2r = h->d_v2r.as<uint32_t>();
      it.real_ptrs = h->d_real_ptrs.as<uint32_t>();
      it.orig_id = h->identity ? nullptr : h->d_orig_id.as<uint32_t>();
      it.levels = levels_out[order[r]];
      it.queue = b->d_queues.as<uint32_t>() + qoff;
      it.n = h->n;
      it.num_vss = h->bvss.num_vss;
      it.src = h->new_id[sources[order[r]]];
      it.pad = 0;
      qoff += 2ull * std::max<uint32_t>(h->bvss.num_vss, 1);
    }
    e = hipMemcpy(b->d_items.p, items.data(), sizeof(ManyItem) * g, hipMemcpyHostToDevice);
    if (e != hipSuccess) return BLEST_ERR_DEVICE;
    *out = b.release();
    return BLEST_OK;
  } catch (const std::bad_alloc&) {
    return BLEST_ERR_OUT_OF_MEMORY;
  } catch (...) {
    return BLEST_ERR_INTERNAL;
  }
}

blest_status blest_batch_run(blest_batch_handle b, void* stream) {
  if (!b) return BLEST_ERR_INVALID_ARGUMENT;
  if (hipSetDevice(b->device) != hipSuccess) return BLEST_ERR_DEVICE;
  hipError_t e = launch_bfs_many(b->d_items.as<ManyItem>(), b->g, b->max_n, b->sigma, b->slots,
                                 static_cast<hipStream_t>(stream));
  return e == hipSuccess ? BLEST_OK : BLEST_ERR_DEVICE;
}

void blest_batch_destroy(blest_batch_handle b) {
  if (!b) return;
  (void)hipSetDevice(b->device);
  delete b;
}

blest_status blest_bfs_many(const blest_handle* hs, const uint32_t* sources, uint32_t g,
                            int32_t* const* levels_out, void* stream) {
  blest_batch* b = nullptr;
  blest_status st = blest_batch_create(hs, sources, g, levels_out, &b);
  if (st != BLEST_OK) return st;
  st = blest_batch_run(b, stream);
  hipEvent_t done = nullptr;
  if (st == BLEST_OK && (hipEventCreateWithFlags(&done, hipEventDisableTiming) != hipSuccess ||
                         hipEventRecord(done, static_cast<hipStream_t>(stream)) != hipSuccess))
    st = BLEST_ERR_DEVICE;
  std::lock_guard<std::mutex> lk(g_pending_mu);
  // free the tables of earlier calls whose launches have finished
  for (size_t i = 0; i < g_pending.size();) {
    if (hipEventQuery(g_pending[i].done) == hipSuccess) {
      (void)hipEventDestroy(g_pending[i].done);
      blest_batch_destroy(g_pending[i].b);
      g_pending[i] = g_pending.back();
      g_pending.pop_back();
    } else {
      ++i;
    }
  }
  if (st == BLEST_OK) {
    g_pending.push_back({b, done});
  } else {
    if (done) (void)hipEventDestroy(done);
    (void)hipDeviceSynchronize();
    blest_batch_destroy(b);
  }
  return st;
}

blest_status blest_configure(blest_handle h, int32_t update, uint32_t block, uint32_t blocks_per_cu, uint32_t group,
                             uint32_t eager_max) {
  if (!h) return BLEST_ERR_INVALID_ARGUMENT;
  blest_options o = h->opt;
  o.update = update;
  o.block = block ? block : 1024;
  o.blocks_per_cu = blocks_per_cu ? blocks_per_cu : 1;
  o.group = group ? group : 2;
  o.eager_max = eager_max;
  if (!valid_options(o)) return BLEST_ERR_INVALID_ARGUMENT;
  const blest_options old = h->opt;
  const int old_mode = h->mode;
  h->opt = o;
  h->mode = mode_of(o.update, h->social, h->u_div_paper);
  if (h->on_device) {
    if (hipSetDevice(h->device) != hipSuccess) return BLEST_ERR_DEVICE;
    blest_status st = set_grid(h);
    if (st != BLEST_OK) {
      h->opt = old;
      h->mode = old_mode;
      (void)set_grid(h);
      return st;
    }
  }
  return BLEST_OK;
}

blest_status blest_stats(blest_handle h, blest_stats_t* o) {
  if (!h || !o) return BLEST_ERR_INVALID_ARGUMENT;
  std::memset(o, 0, sizeof(*o));
  const Bvss& b = h->bvss;
  o->n = h->n;
  o->m = h->m;
  o->sigma = b.sigma;
  o->tau = b.tau;
  o->lanes = 64;
  o->num_slice_sets = b.num_sets;
  o->num_vss = b.num_vss;
  o->num_slices = b.num_slices;
  o->compression = h->compression;
  o->u_div_paper = h->u_div_paper;
  o->u_div_native = h->u_div_native;
  o->social_like = h->social;
  o->reorder_used = h->reorder_used;
  o->update_used = h->mode == 2 ? BLEST_UPDATE_ADAPTIVE : h->mode == 1 ? BLEST_UPDATE_LAZY : BLEST_UPDATE_EAGER;
  o->eager_max = eager_max_of(h);
  o->nranges = h->nranges;
  o->range_len = h->range_len;
  o->bvss_device_bytes = b.num_slices * (4 + b.sigma / 8) + 4ull * (2ull * b.num_vss + 1) + b.num_vss +
                         4ull * (b.num_sets + 1) + (h->identity ? 0 : 4ull * h->n) + (h->packed ? 4 * b.num_slices : 0);
  o->packed = h->packed ? 1 : 0;
  o->multi_ranges = h->multi_ranges;
  o->multi_num_vss = h->multi_ranges > 1 ? h->mpart.num_vss : b.num_vss;
  o->bvss_bytes_table3 = b.num_slices * (4 + b.sigma / 8) + 4ull * (b.num_vss + b.num_sets);
  o->reorder_seconds = h->reorder_seconds;
  o->prepass_used = h->prepass_used;
  o->prepass_seconds = h->prepass_seconds;
  o->window_used = h->window_used;
  o->build_seconds = h->build_seconds;
  o->hubs_sorted = h->hubs_sorted;
  o->grid = h->grid;
  o->block = h->block;
  o->kernel_vgprs = (uint32_t)std::max(h->num_regs, 0);
  o->blocks_per_cu_runtime = h->occ_api;
  o->blocks_per_cu_own = h->occ_own;
  o->lds_bytes = h->mode != 0 ? 4 * h->range_words : 0;
  o->lds_chunk_words = h->mode != 0 && h->range_words ? 1u << h->lds_cshift : 0;
  o->hub_cpos = h->hub_cpos;
  return BLEST_OK;
}

blest_status blest_footprint(blest_handle h, uint32_t k, uint64_t* bytes) {
  if (!h || !bytes || k > 64) return BLEST_ERR_INVALID_ARGUMENT;
  blest_stats_t s;
  blest_stats(h, &s);
  if (k == 0) {
    *bytes = s.bvss_device_bytes;
    return BLEST_OK;
  }
  const uint64_t nw = h->n_words();
  const uint64_t q = 4ull * std::max<uint32_t>(h->bvss.num_vss, 1) * 6;
  uint64_t ws;
  if (k == 1)
    ws = 4 * nw * 4 + 32 * nw + q + kCtrlWords * 4;
  else
    ws = 3ull * h->n * 8 + (uint64_t)h->bvss.num_sets * h->bvss.sigma + q +
         kCtrlWords * 4;  // 64-bit frontier/visited rows, touched bytes
  *bytes = ws + (uint64_t)k * h->n * 4;
  return BLEST_OK;
}

blest_status blest_export(blest_handle h, int32_t which, void* dst, uint64_t cap, uint64_t* size) {
  if (!h || !size) return BLEST_ERR_INVALID_ARGUMENT;
  const void* src = nullptr;
  uint64_t bytes = 0;
  const Bvss& b = h->bvss;
  switch (which) {
    case BLEST_EXPORT_NEW_ID: src = h->new_id.data(); bytes = 4ull * h->new_id.size(); break;
    case BLEST_EXPORT_REAL_PTRS: src = b.real_ptrs.data(); bytes = 4ull * b.real_ptrs.size(); break;
    case BLEST_EXPORT_VIRTUAL_TO_REAL: src = b.v2r.data(); bytes = 4ull * b.v2r.size(); break;
    case BLEST_EXPORT_VSS_BEGIN: src = b.vss_beg.data(); bytes = 4ull * b.vss_beg.size(); break;
    case BLEST_EXPORT_ROW_IDS: src = b.row_ids.data(); bytes = 4ull * b.row_ids.size(); break;
    case BLEST_EXPORT_MASKS: src = b.masks.data(); bytes = b.masks.size(); break;
    case BLEST_EXPORT_VSS_RANGE: src = b.vss_range.data(); bytes = b.vss_range.size(); break;
    case BLEST_EXPORT_ORDER_ID: src = h->order_id.data(); bytes = 4ull * h->order_id.size(); break;
    case BLEST_EXPORT_PREPASS_ID:
      if (h->prepass_id.empty()) {  // identity
        h->prepass_id.resize(h->n);
        for (uint32_t v = 0; v < h->n; ++v) h->prepass_id[v] = v;
      }
      src = h->prepass_id.data();
      bytes = 4ull * h->prepass_id.size();
      break;
    default: return BLEST_ERR_INVALID_ARGUMENT;
  }
  *size = bytes;
  if (dst) std::memcpy(dst, src, std::min(cap, bytes));
  return BLEST_OK;
}

blest_status blest_level_stats(int32_t device, const int32_t* levels, uint32_t k, uint32_t n, uint64_t* reached,
                               uint64_t* total, int32_t* ecc, uint32_t* far, double* closeness, void* stream) {
  if (k == 0) return BLEST_OK;
  if (k > 65535 || (n && !levels) || !reached || !total || !ecc || !far || !closeness)
    return BLEST_ERR_INVALID_ARGUMENT;
  int count = 0;
  if (device < 0 || hipGetDeviceCount(&count) != hipSuccess || device >= count) return BLEST_ERR_NO_DEVICE;
  if (hipSetDevice(device) != hipSuccess) return BLEST_ERR_DEVICE;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus <= 0)
    return BLEST_ERR_DEVICE;
  static_assert(sizeof(unsigned long long) == sizeof(uint64_t), "64-bit counters");
  const hipError_t e = launch_level_stats(levels, k, n, reinterpret_cast<unsigned long long*>(reached),
                                          reinterpret_cast<unsigned long long*>(total), ecc, far, closeness,
                                          (uint32_t)cus, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? BLEST_OK : BLEST_ERR_DEVICE;
}

blest_status blest_model_bytes(blest_handle h, const int32_t* levels, uint32_t k, uint64_t* bytes) {
  if (!h || !levels || !bytes || k == 0 || k > 64) return BLEST_ERR_INVALID_ARGUMENT;
  const Bvss& b = h->bvss;
  const uint32_t n = h->n;
  // Deepest level over all rows; per slice set, the distinct levels present among
  // its vertices in any row (the set is active at iteration l + 1 for each).
  int32_t maxl = 0;
  uint64_t reached = 0;
  for (uint64_t i = 0; i < (uint64_t)k * n; ++i) {
    maxl = std::max(maxl, levels[i]);
    reached += levels[i] >= 0;
  }
  std::vector<uint64_t> lvmask(n, 0);  // bit l: some row has this vertex at level l (l < 64)
  std::vector<uint8_t> deep(n, 0);     // levels >= 64 tracked exactly below
  for (uint32_t j = 0; j < k; ++j)
    for (uint32_t v = 0; v < n; ++v) {
      const int32_t l = levels[(uint64_t)j * n + v];
      if (l < 0) continue;
      if (l < 64) lvmask[h->new_id[v]] |= 1ull << l;
      else deep[h->new_id[v]] = 1;
    }
  const uint64_t per_slice = 4 + b.sigma / 8;
  const uint64_t front = k == 1 ? b.sigma / 8 : 8ull * b.sigma;  // frontier chunk / frontier words of a set
  uint64_t total = 0;
  std::vector<int32_t> seen;
  for (uint32_t s = 0; s < b.num_sets; ++s) {
    const uint32_t nv = b.real_ptrs[s + 1] - b.real_ptrs[s];
    if (nv == 0) continue;
    const uint64_t slices = b.set_beg[s + 1] - b.set_beg[s];
    const uint32_t v0 = s * b.sigma, v1 = std::min<uint32_t>(n, v0 + b.sigma);
    uint64_t m = 0;
    bool any_deep = false;
    for (uint32_t v = v0; v < v1; ++v) {
      m |= lvmask[v];
      any_deep |= deep[v] != 0;
    }
    uint64_t acts = (uint64_t)__builtin_popcountll(m);
    if (any_deep) {  // rare: levels >= 64 (high-diameter graphs), counted exactly
      seen.clear();
      for (uint32_t j = 0; j < k; ++j)
        for (uint32_t v = v0; v < v1; ++v) {
          const int32_t l = levels[(uint64_t)j * n + h->orig_id_of(v)];
          if (l >= 64 && std::find(seen.begin(), seen.end(), l) == seen.end()) seen.push_back(l);
        }
      acts += seen.size();
    }
    total += acts * (slices * per_slice + front + 8ull * nv);
  }
  const uint64_t iters = (uint64_t)maxl + 1;
  if (k == 1) {
    // Stage 2 reads both visited bitmaps at every lazy iteration; the adaptive
    // scheme runs iteration i lazily iff its queue (the VSSs of the sets holding a
    // vertex of level i - 1) has at least eager_max entries
    std::vector<uint64_t> queued(iters + 1, 0);
    for (uint32_t s = 0; s < b.num_sets; ++s) {
      uint64_t m = 0;
      for (uint32_t v = s * b.sigma, v1 = std::min<uint32_t>(n, v + b.sigma); v < v1; ++v) m |= lvmask[v];
      const uint64_t nv = b.real_ptrs[s + 1] - b.real_ptrs[s];
      for (uint32_t l = 0; m && l < 64 && l < iters; ++l)
        if ((m >> l) & 1ull) queued[l + 1] += nv;
    }
    for (uint64_t i = 1; i <= iters; ++i) {
      // levels past 63 are not tracked per set; those iterations are counted as eager
      const bool lazy_iter = h->mode == 1 || (h->mode == 2 && queued[i] >= eager_max_of(h));
      if (lazy_iter) total += 2ull * ((n + 7) / 8);
    }
    total += 4ull * n + 4ull * reached;  // level initialisation + level writes
  } else {
    // Stage 2 per iteration i: a dense iteration (queue >= 1/16 of the VSSs) sweeps
    // every vertex (visited pair, frontier word, state byte: 25 B); a sparse one
    // reads the n state bytes and moves 24 B + 2 state bytes per vertex that
    // changed at level i (one store in Stage 1, one in Stage 2) and zeroes the
    // frontier word of each vertex of level i - 1.  A vertex changes at level l iff
    // some row has it at level l; queues hold the VSSs of sets with such a vertex.
    std::vector<uint64_t> changed(iters + 1, 0), queued(iters + 2, 0);
    std::vector<int32_t> lv;
    std::vector<uint8_t> set_has;
    for (uint32_t s = 0; s < b.num_sets; ++s) {
      const uint32_t v0 = s * b.sigma, v1 = std::min<uint32_t>(n, v0 + b.sigma);
      set_has.assign(iters + 1, 0);
      for (uint32_t v = v0; v < v1; ++v) {
        const uint32_t vo = h->orig_id_of(v);
        lv.clear();
        for (uint32_t j = 0; j < k; ++j) {
          const int32_t l = levels[(uint64_t)j * n + vo];
          if (l >= 0) lv.push_back(l);
        }
        std::sort(lv.begin(), lv.end());
        lv.erase(std::unique(lv.begin(), lv.end()), lv.end());
        for (const int32_t l : lv) {
          ++changed[l];
          set_has[l] = 1;
        }
      }
      const uint64_t nv = b.real_ptrs[s + 1] - b.real_ptrs[s];
      for (uint64_t l = 0; l < iters; ++l)
        if (set_has[l]) queued[l + 1] += nv;
    }
    for (uint64_t i = 1; i <= iters; ++i) {
      if (queued[i] * 16 >= b.num_vss)
        total += 25ull * n;
      else
        total += n + 26ull * (i < iters ? changed[i] : 0) + 8ull * changed[i - 1];
    }
    total += 4ull * k * n + n + 4ull * reached;            // level, visited and state initialisation + level writes
  }
  *bytes = total;
  return BLEST_OK;
}

blest_status blest_server_create(const blest_handle* hs, uint32_t count, uint64_t budget_bytes, uint32_t idle_ms,
                                 blest_server_handle* out) {
  if (!out) return BLEST_ERR_INVALID_ARGUMENT;
  *out = nullptr;
  if (!hs || count == 0 || count > kServeMaxGraphs) return BLEST_ERR_INVALID_ARGUMENT;
  for (uint32_t i = 0; i < count; ++i) {
    if (!hs[i]) return BLEST_ERR_INVALID_ARGUMENT;
    if (!hs[i]->on_device) return BLEST_ERR_NO_DEVICE;
    if (hs[i]->device != hs[0]->device || hs[i]->bvss.sigma != hs[0]->bvss.sigma ||
        hs[i]->bvss.slots != hs[0]->bvss.slots)
      return BLEST_ERR_INVALID_ARGUMENT;
    if (hs[i]->bvss.num_vss > 0x7FFFFFFFu / 2 || hs[i]->bvss.num_sets >= (1u << 28)) return BLEST_ERR_TOO_LARGE;
  }
  try {
    std::unique_ptr<blest_server> sv(new blest_server);
    sv->device = hs[0]->device;
    if (hipSetDevice(sv->device) != hipSuccess) return BLEST_ERR_DEVICE;
    sv->sigma = hs[0]->bvss.sigma;
    sv->slots = hs[0]->bvss.slots;
    sv->budget = budget_bytes;
    sv->idle_limit = (idle_ms ? idle_ms : 20) * 100000u;  // s_memrealtime runs at 100 MHz
    hipError_t e = hipSuccess;
    for (uint32_t i = 0; i < count && e == hipSuccess; ++i) {
      blest_graph* h = hs[i];
      sv->graphs.push_back(h);
      auto st = std::make_unique<blest_server::GraphState>();
      const uint64_t qcap = 2ull * std::max<uint32_t>(h->bvss.num_vss, 1);
      e = st->vis.alloc(16ull * h->n);
      if (e == hipSuccess) e = st->front.alloc(8ull * h->n);
      if (e == hipSuccess) e = st->touched.alloc((uint64_t)std::max<uint32_t>(h->bvss.num_sets, 1) * h->bvss.sigma);
      if (e == hipSuccess) e = st->queue.alloc(2 * 4 * qcap);
      if (e == hipSuccess) e = hipMemset(st->vis.p, 0, st->vis.bytes);
      if (e == hipSuccess) e = hipMemset(st->front.p, 0, st->front.bytes);
      if (e == hipSuccess) e = hipMemset(st->touched.p, 0, st->touched.bytes);
      sv->resident += st->vis.bytes + st->front.bytes + st->touched.bytes + st->queue.bytes;
      sv->gs.push_back(std::move(st));
    }
    if (e == hipSuccess) e = sv->state.alloc(sizeof(ServeState));
    if (e == hipSuccess) e = hipMemset(sv->state.p, 0, sizeof(ServeState));
    if (e == hipSuccess) {
      const uint32_t one = 1;  // iterations are numbered from 1
      e = hipMemcpy(reinterpret_cast<char*>(sv->state.p) + offsetof(ServeState, iter), &one, 4,
                    hipMemcpyHostToDevice);
    }
    if (e == hipSuccess) e = sv->ctrl.alloc(4ull * kServeCtrlWords);
    if (e == hipSuccess) e = hipMemset(sv->ctrl.p, 0, 4ull * kServeCtrlWords);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&sv->mb), sizeof(ServeMailbox),
                                           hipHostMallocCoherent | hipHostMallocMapped);
    if (e == hipSuccess) {
      std::memset(sv->mb, 0, sizeof(ServeMailbox));
      e = hipHostGetDevicePointer(reinterpret_cast<void**>(&sv->mb_dev), sv->mb, 0);
    }
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&sv->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&sv->ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) return e == hipErrorOutOfMemory ? BLEST_ERR_OUT_OF_MEMORY : BLEST_ERR_DEVICE;
    sv->resident += sizeof(ServeState) + 4ull * kServeCtrlWords;
    const void* k = serve_kernel_symbol(sv->sigma, sv->slots);
    int cus = 0, nb = 0, regs = 0;
    if (!k || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, sv->device) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, (int)sv->block, 0) != hipSuccess || nb <= 0)
      return BLEST_ERR_DEVICE;
    const uint32_t own = own_blocks_per_cu(k, sv->block, 0, &regs);
    sv->grid = std::min<uint32_t>({(uint32_t)nb, own, 1u}) * (uint32_t)cus;
    if (sv->grid == 0) return BLEST_ERR_DEVICE;
    *out = sv.release();
    return BLEST_OK;
  } catch (const std::bad_alloc&) {
    return BLEST_ERR_OUT_OF_MEMORY;
  } catch (...) {
    return BLEST_ERR_INTERNAL;
  }
}

blest_status blest_server_submit(blest_server_handle sv, uint32_t graph, const uint32_t* sources, uint32_t k,
                                 int32_t* levels_out, uint64_t* ticket) {
  if (!sv || !sources || !levels_out || !ticket || graph >= sv->graphs.size() || k == 0 || k > kServeCols)
    return BLEST_ERR_INVALID_ARGUMENT;
  const blest_graph* h = sv->graphs[graph];
  for (uint32_t j = 0; j < k; ++j)
    if (sources[j] >= h->n) return BLEST_ERR_INVALID_ARGUMENT;
  try {
    std::lock_guard<std::mutex> lk(sv->mu);
    const uint64_t bytes = 4ull * k * h->n;
    const uint32_t r = sv->next_ticket % kServeRing;
    ServeSlot* slot = &sv->mb->slot[r];
    if (sv->outstanding + bytes > sv->budget ||
        __atomic_load_n(&slot->state, __ATOMIC_ACQUIRE) != 0)  // ring slot still held by an unreleased request
      return BLEST_ERR_BUDGET;
    slot->graph = graph;
    slot->k = k;
    slot->admit_iter = slot->done_iter = slot->levels = 0;
    slot->out = reinterpret_cast<uint64_t>(levels_out);
    for (uint32_t j = 0; j < k; ++j) slot->src[j] = h->new_id[sources[j]];
    __atomic_store_n(&slot->state, 1u, __ATOMIC_RELAXED);
    __atomic_store_n(&sv->mb->submitted, sv->next_ticket + 1, __ATOMIC_RELEASE);
    *ticket = sv->next_ticket++;
    sv->charge[r] = bytes;
    sv->outstanding += bytes;
    sv->peak = std::max(sv->peak, sv->outstanding);
    return server_ensure_running(sv) == hipSuccess ? BLEST_OK : BLEST_ERR_DEVICE;
  } catch (...) {
    return BLEST_ERR_INTERNAL;
  }
}

blest_status blest_server_poll(blest_server_handle sv, uint64_t ticket, int32_t* state, uint32_t* levels,
                               uint32_t* admit_iter, uint32_t* done_iter) {
  if (!sv || !state) return BLEST_ERR_INVALID_ARGUMENT;
  std::lock_guard<std::mutex> lk(sv->mu);
  if (ticket >= sv->next_ticket || sv->next_ticket - ticket > kServeRing) return BLEST_ERR_INVALID_ARGUMENT;
  const ServeSlot* slot = &sv->mb->slot[ticket % kServeRing];
  const uint32_t s = __atomic_load_n(&slot->state, __ATOMIC_ACQUIRE);
  if (s == 0) return BLEST_ERR_INVALID_ARGUMENT;  // released
  *state = (int32_t)s - 1;                        // 0 waiting, 1 running, 2 done
  if (levels) *levels = slot->levels;
  if (admit_iter) *admit_iter = slot->admit_iter;
  if (done_iter) *done_iter = slot->done_iter;
  // a launch that ended (idle limit) just before this request was published is
  // followed by a new one
  if (s == 1 && server_ensure_running(sv) != hipSuccess) return BLEST_ERR_DEVICE;
  return BLEST_OK;
}

blest_status blest_server_release(blest_server_handle sv, uint64_t ticket) {
  if (!sv) return BLEST_ERR_INVALID_ARGUMENT;
  std::lock_guard<std::mutex> lk(sv->mu);
  if (ticket >= sv->next_ticket || sv->next_ticket - ticket > kServeRing) return BLEST_ERR_INVALID_ARGUMENT;
  const uint32_t r = ticket % kServeRing;
  ServeSlot* slot = &sv->mb->slot[r];
  if (__atomic_load_n(&slot->state, __ATOMIC_ACQUIRE) != 3) return BLEST_ERR_INVALID_ARGUMENT;
  __atomic_store_n(&slot->state, 0u, __ATOMIC_RELEASE);
  sv->outstanding -= sv->charge[r];
  sv->charge[r] = 0;
  return BLEST_OK;
}

blest_status blest_server_stats(blest_server_handle sv, blest_server_stats_t* out) {
  if (!sv || !out) return BLEST_ERR_INVALID_ARGUMENT;
  std::lock_guard<std::mutex> lk(sv->mu);
  std::memset(out, 0, sizeof(*out));
  out->budget = sv->budget;
  out->outstanding = sv->outstanding;
  out->peak_outstanding = sv->peak;
  out->resident_bytes = sv->resident;
  out->submitted = sv->next_ticket;
  out->launches = sv->launches;
  out->running = sv->launched && hipEventQuery(sv->ev) == hipErrorNotReady;
  out->grid = sv->grid;
  out->block = sv->block;
  // the mailbox is coherent host memory; the kernel writes these when a launch ends
  volatile const uint64_t* prof = sv->mb->prof;
  out->iterations = prof[4];
  out->control_us = prof[0] * 0.01;  // 100 MHz realtime ticks
  out->stage1_us = prof[1] * 0.01;
  out->stage2_us = prof[2] * 0.01;
  out->admit_us = prof[3] * 0.01;
  return BLEST_OK;
}

blest_status blest_server_destroy(blest_server_handle sv, uint32_t timeout_ms) {
  if (!sv) return BLEST_OK;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    __atomic_store_n(&sv->mb->stop, 1u, __ATOMIC_RELEASE);
  }
  // the launch ends once nothing waits or runs; past the time limit it is told to
  // end at its next level boundary (stop = 2), running requests or not
  const double limit = (timeout_ms ? timeout_ms : 60000) / 1000.0;
  double t0 = now_s();
  bool aborted = false;
  while (sv->launched && hipEventQuery(sv->ev) == hipErrorNotReady) {
    if (now_s() - t0 > limit) {
      if (aborted) return BLEST_ERR_DEVICE;  // still running: nothing freed
      __atomic_store_n(&sv->mb->stop, 2u, __ATOMIC_RELEASE);
      aborted = true;
      t0 = now_s();
    }
    std::this_thread::sleep_for(std::chrono::microseconds(200));
  }
  (void)hipSetDevice(sv->device);
  delete sv;
  return BLEST_OK;
}

blest_status blest_barrier_probe(int32_t device, uint32_t block, uint32_t max_grid, uint32_t rounds,
                                 double* seconds_per_barrier) {
  if (!seconds_per_barrier || rounds == 0 || block == 0 || block % 64 != 0 || block > 1024)
    return BLEST_ERR_INVALID_ARGUMENT;
  int count = 0;
  if (device < 0 || hipGetDeviceCount(&count) != hipSuccess || device >= count) return BLEST_ERR_NO_DEVICE;
  if (hipSetDevice(device) != hipSuccess) return BLEST_ERR_DEVICE;
  int cus = 0, nb = 0, regs = 0;
  const void* k = barrier_probe_symbol();
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, (int)block, 0) != hipSuccess || nb <= 0)
    return BLEST_ERR_DEVICE;
  // one workgroup per CU, as the BFS launches of that workgroup size
  uint32_t grid = std::min<uint32_t>({(uint32_t)nb, own_blocks_per_cu(k, block, 0, &regs), 1u}) * (uint32_t)cus;
  if (max_grid && grid > max_grid) grid = max_grid;
  DevBuf ctrl;
  hipEvent_t a = nullptr, b = nullptr;
  hipError_t e = ctrl.alloc(4ull * kCtrlWords);
  if (e == hipSuccess) e = hipMemset(ctrl.p, 0, 4ull * kCtrlWords);
  if (e == hipSuccess) e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  float ms[2] = {0, 0};
  for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {  // the first run warms up
    if (e == hipSuccess) e = hipEventRecord(a, nullptr);
    if (e == hipSuccess) e = launch_barrier_probe(ctrl.as<uint32_t>(), rounds, grid, block, nullptr);
    if (e == hipSuccess) e = hipEventRecord(b, nullptr);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms[rep], a, b);
  }
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  if (e != hipSuccess) return BLEST_ERR_DEVICE;
  *seconds_per_barrier = ms[1] / 1000.0 / rounds;
  return BLEST_OK;
}

void blest_shutdown(void) {
  {
    std::lock_guard<std::mutex> lk(g_pending_mu);
    for (PendingBatch& pb : g_pending) {
      (void)hipEventSynchronize(pb.done);
      (void)hipEventDestroy(pb.done);
      blest_batch_destroy(pb.b);
    }
    g_pending.clear();
  }
  for (int d = 0; d < 64; ++d) {
    DeviceSerial& ds = g_serial[d];
    std::lock_guard<std::mutex> lk(ds.mu);
    if (!ds.last) continue;
    (void)hipEventSynchronize(ds.last);
    (void)hipEventDestroy(ds.last);
    ds.last = nullptr;
  }
}

void blest_destroy(blest_handle h) {
  if (!h) return;
  if (h->on_device) (void)hipSetDevice(h->device);
  delete h;
}

const char* blest_status_string(blest_status s) {
  switch (s) {
    case BLEST_OK: return "ok";
    case BLEST_ERR_INVALID_ARGUMENT: return "invalid argument";
    case BLEST_ERR_INVALID_GRAPH: return "invalid graph";
    case BLEST_ERR_TOO_LARGE: return "graph too large (nnz >= 2^32)";
    case BLEST_ERR_OUT_OF_MEMORY: return "out of memory";
    case BLEST_ERR_BUDGET: return "device budget exceeded";
    case BLEST_ERR_DEVICE: return "device error";
    case BLEST_ERR_NO_DEVICE: return "no device (host-only handle or no GPU)";
    case BLEST_ERR_INTERNAL: return "internal error";
  }
  return "unknown status";
}

}  // extern "C"
