// Seeded synthetic graph inputs shared by the oracle, the tests and the benchmark.
//
// This file holds no part of the BFS method: it only draws graphs and sources and
// normalises them into a CSR (sorted neighbour lists, no self-loops, no duplicate
// arcs).  Both the oracle and the GPU library consume its output, so nothing here
// may compute levels, slices or orderings.
//
// Randomness is counter based: every random number is splitmix64(stream, counter),
// with the splitmix64 output function of Steele, Lea and Flood ("Fast splittable
// pseudorandom number generators", OOPSLA 2014).  A draw therefore depends only on
// (seed, stream tag, counter), never on thread scheduling.
//
// Generators:
//   R-MAT (Chakrabarti, Zhan, Faloutsos 2004) with initiator (a, b, c, d), no
//   noise: draw e picks one quadrant per bit level, top bit first, from the
//   uniform 32-bit number u = half (level & 1) of splitmix64(seed_rmat, e*ceil(S/2)
//   + level/2); quadrant 0 if u < a*2^32, 1 if u < (a+b)*2^32, 2 if u < (a+b+c)*2^32,
//   else 3.  Quadrant q sets row bit (q >> 1) and column bit (q & 1).
//   Grid R x C: vertex (r, c) is r*C + c; the right edge of v is kept iff
//   U(seed_grid, 2v) < p, the down edge iff U(seed_grid, 2v+1) < p, where U is the
//   top 53 bits of splitmix64 scaled to [0, 1).
// Every generator symmetrises, drops self-loops and removes duplicate arcs.

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <new>
#include <thread>
#include <vector>

namespace {

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;

inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Stream key for (seed, tag): a mixed seed so that different tags never share draws.
inline uint64_t stream_key(uint64_t seed, uint64_t tag) { return mix64(seed ^ mix64(tag * kGamma + 1)); }

inline uint64_t draw(uint64_t key, uint64_t counter) { return mix64(key + (counter + 1) * kGamma); }

inline double unit53(uint64_t z) { return (double)(z >> 11) * (1.0 / 9007199254740992.0); }

inline uint64_t mulhi64(uint64_t a, uint64_t b) { return (uint64_t)(((unsigned __int128)a * b) >> 64); }

enum : uint64_t { kTagRmat = 1, kTagGrid = 2, kTagPerm = 3, kTagSrc = 4 };

int hw_threads() {
  const char* s = std::getenv("GG_THREADS");
  if (s && std::atoi(s) > 0) return std::atoi(s);
  unsigned h = std::thread::hardware_concurrency();
  if (h == 0) h = 1;
  return (int)std::min<unsigned>(h, 16);
}

template <class F>
void parallel_for(uint64_t n, F&& body) {
  int T = hw_threads();
  if (n < 100000 || T == 1) {
    body(0, n);
    return;
  }
  std::vector<std::thread> th;
  uint64_t chunk = (n + T - 1) / T;
  for (int t = 0; t < T; ++t) {
    uint64_t lo = t * chunk, hi = std::min<uint64_t>(n, lo + chunk);
    if (lo >= hi) break;
    th.emplace_back([&, lo, hi] { body(lo, hi); });
  }
  for (auto& x : th) x.join();
}

// Large uninitialised buffer whose pages are first touched by all threads (first
// touch from a single thread is several times slower on big graphs).
struct Buf {
  uint32_t* p = nullptr;
  uint64_t n = 0;
  Buf() = default;
  explicit Buf(uint64_t count) : p(static_cast<uint32_t*>(std::malloc(sizeof(uint32_t) * (count ? count : 1)))), n(count) {
    if (!p) throw std::bad_alloc();
    parallel_for(count, [&](uint64_t lo, uint64_t hi) { std::memset(p + lo, 0, sizeof(uint32_t) * (hi - lo)); });
  }
  Buf(const Buf&) = delete;
  Buf& operator=(const Buf&) = delete;
  Buf(Buf&& o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
  Buf& operator=(Buf&& o) noexcept { std::swap(p, o.p); std::swap(n, o.n); return *this; }
  ~Buf() { std::free(p); }
  uint32_t* data() { return p; }
  const uint32_t* data() const { return p; }
  uint32_t& operator[](uint64_t i) { return p[i]; }
  const uint32_t& operator[](uint64_t i) const { return p[i]; }
  uint64_t size() const { return n; }
};

struct Csr {
  uint32_t n = 0;
  Buf row_ptr;  // n + 1
  Buf col;      // nnz
};

// Builds a normalised CSR from an arc list (src[i] -> dst[i]).  With symmetrise the
// reverse arc is added as well.  Self-loops and duplicates are removed and every
// neighbour list is sorted.  Each thread owns a contiguous range of rows and scans
// the whole arc list, so no atomics are needed and the result does not depend on
// the thread count.
Csr* csr_from_arcs(uint32_t n, uint64_t m, const uint32_t* src, const uint32_t* dst, bool symmetrise) {
  Csr* g = new Csr;
  g->n = n;
  int T = (m < 100000) ? 1 : hw_threads();
  std::vector<uint64_t> ptr(n + 1, 0);
  auto for_ranges = [&](auto&& body) {
    std::vector<std::thread> th;
    uint64_t chunk = ((uint64_t)n + T - 1) / T;
    for (int t = 0; t < T; ++t) {
      uint32_t lo = (uint32_t)std::min<uint64_t>(n, t * chunk);
      uint32_t hi = (uint32_t)std::min<uint64_t>(n, lo + chunk);
      if (T == 1) { body(lo, hi); return; }
      th.emplace_back([&, lo, hi] { body(lo, hi); });
    }
    for (auto& x : th) x.join();
  };
  // Pass 1: degree counts (ptr[v + 1] holds the count of row v).
  for_ranges([&](uint32_t lo, uint32_t hi) {
    for (uint64_t i = 0; i < m; ++i) {
      uint32_t s = src[i], d = dst[i];
      if (s == d) continue;
      if (s >= lo && s < hi) ++ptr[s + 1];
      if (symmetrise && d >= lo && d < hi) ++ptr[d + 1];
    }
  });
  for (uint32_t v = 0; v < n; ++v) ptr[v + 1] += ptr[v];
  Buf tmp(ptr[n]);
  // Pass 2: scatter arcs into their rows.
  for_ranges([&](uint32_t lo, uint32_t hi) {
    std::vector<uint64_t> cur(ptr.begin() + lo, ptr.begin() + hi);
    for (uint64_t i = 0; i < m; ++i) {
      uint32_t s = src[i], d = dst[i];
      if (s == d) continue;
      if (s >= lo && s < hi) tmp[cur[s - lo]++] = d;
      if (symmetrise && d >= lo && d < hi) tmp[cur[d - lo]++] = s;
    }
  });
  // Sort and deduplicate each row in place; record the unique count.
  std::vector<uint32_t> uniq(n, 0);
  {
    std::atomic<uint64_t> next(0);
    const uint64_t step = 4096;
    std::vector<std::thread> th;
    auto work = [&] {
      for (;;) {
        uint64_t lo = next.fetch_add(step);
        if (lo >= n) break;
        uint64_t hi = std::min<uint64_t>(n, lo + step);
        for (uint64_t v = lo; v < hi; ++v) {
          uint32_t* b = tmp.data() + ptr[v];
          uint32_t* e = tmp.data() + ptr[v + 1];
          std::sort(b, e);
          uniq[v] = (uint32_t)(std::unique(b, e) - b);
        }
      }
    };
    for (int t = 1; t < T; ++t) th.emplace_back(work);
    work();
    for (auto& x : th) x.join();
  }
  g->row_ptr = Buf((uint64_t)n + 1);
  uint64_t acc = 0;
  for (uint32_t v = 0; v < n; ++v) {
    acc += uniq[v];
    if (acc > 0xFFFFFFFFull) {  // the CSR holds 32-bit offsets
      delete g;
      return nullptr;
    }
    g->row_ptr[v + 1] = (uint32_t)acc;
  }
  g->col = Buf(acc);
  parallel_for(n, [&](uint64_t lo, uint64_t hi) {
    for (uint64_t v = lo; v < hi; ++v)
      std::memcpy(g->col.data() + g->row_ptr[v], tmp.data() + ptr[v], sizeof(uint32_t) * uniq[v]);
  });
  return g;
}

}  // namespace

extern "C" {

// R-MAT graph with 2^scale vertices and ef * 2^scale edge draws, symmetrised.
void* gg_rmat(int scale, int ef, double a, double b, double c, uint64_t seed) {
  if (scale < 1 || scale > 31 || ef < 1) return nullptr;
  uint32_t n = 1u << scale;
  uint64_t m = (uint64_t)ef << scale;
  uint64_t key = stream_key(seed, kTagRmat);
  const double two32 = 4294967296.0;
  uint64_t ta = (uint64_t)std::llround(a * two32);
  uint64_t tab = (uint64_t)std::llround((a + b) * two32);
  uint64_t tabc = (uint64_t)std::llround((a + b + c) * two32);
  uint64_t per_edge = (uint64_t)(scale + 1) / 2;
  Buf src(m), dst(m);
  parallel_for(m, [&](uint64_t lo, uint64_t hi) {
    for (uint64_t e = lo; e < hi; ++e) {
      uint32_t r = 0, cc = 0;
      uint64_t z = 0;
      for (int level = 0; level < scale; ++level) {
        if ((level & 1) == 0) z = draw(key, e * per_edge + (uint64_t)(level >> 1));
        uint64_t u = (level & 1) ? (z >> 32) : (z & 0xFFFFFFFFull);
        uint32_t q = u < ta ? 0u : u < tab ? 1u : u < tabc ? 2u : 3u;
        int bit = scale - 1 - level;
        r |= (q >> 1) << bit;
        cc |= (q & 1u) << bit;
      }
      src[e] = r;
      dst[e] = cc;
    }
  });
  return csr_from_arcs(n, m, src.data(), dst.data(), true);
}

// R x C four-neighbour grid; each right/down edge kept with probability p.
void* gg_grid(uint32_t R, uint32_t C, double p, uint64_t seed) {
  uint64_t n64 = (uint64_t)R * C;
  if (R == 0 || C == 0 || n64 > 0xFFFFFFFFull) return nullptr;
  uint32_t n = (uint32_t)n64;
  uint64_t key = stream_key(seed, kTagGrid);
  // Upper bound on kept edges: 2 per vertex.
  std::vector<uint32_t> src, dst;
  src.reserve(2 * n64);
  dst.reserve(2 * n64);
  for (uint32_t r = 0; r < R; ++r)
    for (uint32_t c = 0; c < C; ++c) {
      uint32_t v = r * C + c;
      if (c + 1 < C && unit53(draw(key, 2ull * v)) < p) {
        src.push_back(v);
        dst.push_back(v + 1);
      }
      if (r + 1 < R && unit53(draw(key, 2ull * v + 1)) < p) {
        src.push_back(v);
        dst.push_back(v + C);
      }
    }
  return csr_from_arcs(n, src.size(), src.data(), dst.data(), true);
}

// CSR from an explicit arc list; symmetrise != 0 adds reverse arcs.
void* gg_from_arcs(uint32_t n, uint64_t m, const uint32_t* src, const uint32_t* dst, int symmetrise) {
  for (uint64_t i = 0; i < m; ++i)
    if (src[i] >= n || dst[i] >= n) return nullptr;
  return csr_from_arcs(n, m, src, dst, symmetrise != 0);
}

// Seeded uniform permutation of 0..n-1 (Fisher-Yates, Lemire's multiply-high
// reduction of each 64-bit draw onto [0, i]).
void gg_permutation(uint32_t n, uint64_t seed, uint32_t* perm) {
  for (uint32_t i = 0; i < n; ++i) perm[i] = i;
  uint64_t key = stream_key(seed, kTagPerm);
  for (uint32_t i = n; i > 1; --i) {
    uint32_t j = (uint32_t)mulhi64(draw(key, i - 1), i);
    std::swap(perm[i - 1], perm[j]);
  }
}

// Relabels a CSR: vertex v becomes perm[v].  Rows stay normalised (sorted); the
// input must already be free of self-loops and duplicates, which relabelling keeps.
void* gg_relabel(uint32_t n, const uint32_t* row_ptr, const uint32_t* col, const uint32_t* perm) {
  std::vector<uint32_t> inv(n);
  for (uint32_t v = 0; v < n; ++v) {
    if (perm[v] >= n) return nullptr;
    inv[perm[v]] = v;
  }
  Csr* g = new Csr;
  g->n = n;
  g->row_ptr = Buf((uint64_t)n + 1);
  uint64_t acc = 0;
  for (uint32_t w = 0; w < n; ++w) {
    acc += row_ptr[inv[w] + 1] - row_ptr[inv[w]];
    g->row_ptr[w + 1] = (uint32_t)acc;
  }
  g->col = Buf(acc);
  parallel_for(n, [&](uint64_t lo, uint64_t hi) {
    for (uint64_t w = lo; w < hi; ++w) {
      uint32_t v = inv[w];
      uint32_t* out = g->col.data() + g->row_ptr[w];
      uint32_t d = row_ptr[v + 1] - row_ptr[v];
      for (uint32_t i = 0; i < d; ++i) out[i] = perm[col[row_ptr[v] + i]];
      std::sort(out, out + d);
    }
  });
  return g;
}

// k sources drawn uniformly among vertices with out-degree > 0.  distinct != 0
// rejects repeats (counter keeps advancing).  Returns the number written; fewer than
// k only if distinct is requested and fewer candidates exist.
uint32_t gg_sources(uint32_t n, const uint32_t* row_ptr, uint64_t seed, uint32_t k, int distinct,
                    uint32_t* out) {
  std::vector<uint32_t> cand;
  for (uint32_t v = 0; v < n; ++v)
    if (row_ptr[v + 1] > row_ptr[v]) cand.push_back(v);
  if (cand.empty()) return 0;
  if (distinct && k > cand.size()) k = (uint32_t)cand.size();
  uint64_t key = stream_key(seed, kTagSrc);
  std::vector<char> used(distinct ? n : 0, 0);
  uint32_t got = 0;
  for (uint64_t t = 0; got < k; ++t) {
    uint32_t v = cand[mulhi64(draw(key, t), cand.size())];
    if (distinct) {
      if (used[v]) continue;
      used[v] = 1;
    }
    out[got++] = v;
  }
  return got;
}

// Raw counter-based draws, exposed so tests can pin the generator.
uint64_t gg_draw(uint64_t seed, uint64_t tag, uint64_t counter) { return draw(stream_key(seed, tag), counter); }

uint32_t gg_n(const void* h) { return static_cast<const Csr*>(h)->n; }
uint64_t gg_nnz(const void* h) { return static_cast<const Csr*>(h)->col.size(); }
void gg_copy(const void* h, uint32_t* row_ptr, uint32_t* col) {
  const Csr* g = static_cast<const Csr*>(h);
  std::memcpy(row_ptr, g->row_ptr.data(), sizeof(uint32_t) * (g->n + 1));
  parallel_for(g->col.size(), [&](uint64_t lo, uint64_t hi) {
    std::memcpy(col + lo, g->col.data() + lo, sizeof(uint32_t) * (hi - lo));
  });
}
void gg_free(void* h) { delete static_cast<Csr*>(h); }

}  // extern "C"
