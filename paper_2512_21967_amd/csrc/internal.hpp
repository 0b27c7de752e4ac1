// Internal declarations shared by the host-side builder (host.cpp), the HIP kernels
// (kernels.hip) and the C-ABI (capi.cpp).  Not part of the public interface.
#pragma once

#include <cstdint>
#include <vector>

namespace blest {

// Out-neighbour CSR with sorted, duplicate-free rows and no self-loops.
struct Csr {
  uint32_t n = 0;
  std::vector<uint32_t> rp;   // n + 1
  std::vector<uint32_t> col;  // rp[n]
  uint64_t nnz() const { return rp.empty() ? 0 : rp.back(); }
};

// Result codes of the host helpers (mapped onto blest_status by the C-ABI).
enum HostRc { kOk = 0, kInvalidGraph = 2, kTooLarge = 3, kNoMemory = 4 };

// Validates a caller CSR and writes its normal form (loops and duplicates dropped,
// rows sorted).
int normalise(uint32_t n, uint64_t nnz, const uint32_t* rp, const uint32_t* col, int threads, Csr& out);

// In-neighbour CSR (the transposed graph).
void transpose(const Csr& g, Csr& t);

// Undirected view: N(v) = out(v) union in(v).
void undirected(const Csr& g, const Csr& gt, Csr& u);

// Vertex v gets label new_id[v]; rows stay sorted.
void relabel(const Csr& g, const std::vector<uint32_t>& new_id, int threads, Csr& out);

// Social-like test of Section 2.2.1 (heavy tail or power-law fit).
bool social_like(const Csr& g);

// Algorithm 1 (JaccardWithWindows).  gt is the in-neighbour CSR.  Output: new_id.
void jaccard_windows(const Csr& g, const Csr& gt, uint32_t sigma, uint32_t w, int threads,
                     std::vector<uint32_t>& new_id);

// Shingle ordering (Chierichetti et al., "On compressing social networks", KDD
// 2009), the locality pre-pass run before Algorithm 1 in place of Gorder
// (Section 2.2 names Gorder without specifying it): vertex v gets the key
// (min over out-neighbours u of h_0(u), ..., of h_{k-1}(u)) and vertices take labels
// in ascending key order, ties by ID; no out-neighbours: every component is
// 2^64 - 1.  h_i(u) is output u + 1 of the SplitMix64 stream (Steele, Lea and
// Flood, OOPSLA 2014) seeded with s_i, and s_i is output i + 1 of the stream
// seeded with `seed`.  Output: new_id.
void shingle_order(const Csr& g, uint32_t hashes, uint64_t seed, int threads, std::vector<uint32_t>& new_id);
uint64_t splitmix64(uint64_t seed, uint64_t t);  // output t (t >= 1) of the stream seeded with seed

// Reverse Cuthill-McKee on the undirected view u.  Output: new_id.
void rcm(const Csr& u, std::vector<uint32_t>& new_id);

// Reorders sigma-aligned vertex groups by summed in-degree (largest first), keeping
// each group intact, and places the hottest words at the first cpos positions of
// every 64-word chunk (cpos = 0: plain rank order).  Output: new_id.
void hub_sort(const Csr& g, uint32_t sigma, uint32_t cpos, std::vector<uint32_t>& new_id);

// LDS cache of one row range of rw visited words: the first C = 2^cshift (<= 64)
// words of every 64-word chunk, C as large as cap_words allows.  Returns the
// cached word count (0 when not even one word per chunk fits).
inline uint32_t cache_shape(uint32_t rw, uint32_t cap_words, uint32_t& cshift) {
  const uint32_t chunks = (rw + 63) / 64;
  cshift = 0;
  if (chunks == 0 || cap_words < chunks) return 0;
  const uint32_t per = cap_words / chunks;
  while (cshift < 6 && (2u << cshift) <= per) ++cshift;
  return chunks << cshift;
}

// The static BVSS arrays (Section 2.1) in this library's layout: the slices of a
// slice set are sorted by row and cut into VSSs of at most tau = 64 * slots, a cut
// also falling at every multiple of range_len in row ID (when range_len > 0) so
// that each VSS pulls rows of one row range only; VSS v owns slices
// [vss_beg[v], vss_beg[v+1]) stored contiguously, so lane l of a wavefront handles
// slices l, l + 64, ... of the VSS (column-major placement, Section 2.1.2) and
// nothing is padded.
struct Bvss {
  uint32_t n = 0, sigma = 8, slots = 4, tau = 256, range_len = 0;
  uint32_t num_sets = 0, num_vss = 0;
  uint64_t num_slices = 0;
  std::vector<uint32_t> real_ptrs;  // num_sets + 1
  std::vector<uint32_t> v2r;        // num_vss
  std::vector<uint32_t> vss_beg;    // num_vss + 1
  std::vector<uint32_t> set_beg;    // num_sets + 1 (first slice of each set)
  std::vector<uint8_t> vss_range;   // num_vss: row range of each VSS
  std::vector<uint32_t> row_ids;    // num_slices
  std::vector<uint8_t> masks;       // num_slices * sigma / 8
  uint32_t mask_bytes() const { return sigma / 8; }
  uint64_t mask_of(uint64_t k) const {
    uint64_t m = 0;
    for (uint32_t b = 0; b < sigma / 8; ++b) m |= (uint64_t)masks[k * (sigma / 8) + b] << (8 * b);
    return m;
  }
};

// A VSS partition of a Bvss's slices (the arrays of the same names in Bvss).
struct VssPartition {
  uint32_t num_vss = 0, range_len = 0;
  std::vector<uint32_t> real_ptrs, v2r, vss_beg;
  std::vector<uint8_t> vss_range;
};

// Slices of every set (set_beg, row_ids, masks); then the VSS partition.
int build_slices(const Csr& g, uint32_t sigma, uint32_t slots, int threads, Bvss& out);
int partition_vss(Bvss& b, uint32_t range_len, int threads);
// The same partition into separate arrays (b is not changed).
void partition_vss_into(const Bvss& b, uint32_t range_len, int threads, VssPartition& out);

// Update divergence (Section 2.2.1) when each set's sorted slices are cut into
// VSSs of lanes * slots_per_lane and columns of `lanes` consecutive slices;
// slots_per_lane = 0 uses this layout's own VSSs.
double update_divergence(const Bvss& b, uint32_t lanes, uint32_t slots_per_lane);

}  // namespace blest
