// Host-side preprocessing: CSR normalisation, the two orderings of Section 2.2
// (Algorithm 1 and reverse Cuthill-McKee), the social-like test of Section 2.2.1,
// and construction of the BVSS arrays of Section 2.1.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <functional>
#include <numeric>
#include <thread>

#include "internal.hpp"

namespace blest {
namespace {

int pick_threads(int threads) {
  if (threads > 0) return threads;
  unsigned h = std::thread::hardware_concurrency();
  return h == 0 ? 1 : (int)std::min<unsigned>(h, 64);
}

// Runs body(lo, hi) over [0, n) in dynamically claimed chunks.
void parallel_chunks(uint64_t n, uint64_t chunk, int threads, const std::function<void(uint64_t, uint64_t)>& body) {
  int T = pick_threads(threads);
  if (T <= 1 || n <= chunk) {
    if (n) body(0, n);
    return;
  }
  std::atomic<uint64_t> next(0);
  auto work = [&] {
    for (;;) {
      uint64_t lo = next.fetch_add(chunk);
      if (lo >= n) return;
      body(lo, std::min(n, lo + chunk));
    }
  };
  std::vector<std::thread> th;
  for (int t = 1; t < T; ++t) th.emplace_back(work);
  work();
  for (auto& x : th) x.join();
}

}  // namespace

int normalise(uint32_t n, uint64_t nnz, const uint32_t* rp, const uint32_t* col, int threads, Csr& out) {
  if (nnz > 0xFFFFFFFFull) return kTooLarge;
  if (rp[0] != 0 || rp[n] != nnz) return kInvalidGraph;
  for (uint32_t v = 0; v < n; ++v)
    if (rp[v + 1] < rp[v]) return kInvalidGraph;
  std::atomic<bool> bad(false);
  std::vector<uint32_t> keep(n, 0);
  std::vector<uint32_t> tmp(nnz);
  parallel_chunks(n, 4096, threads, [&](uint64_t lo, uint64_t hi) {
    for (uint64_t v = lo; v < hi; ++v) {
      uint32_t* b = tmp.data() + rp[v];
      uint32_t d = 0;
      for (uint32_t i = rp[v]; i < rp[v + 1]; ++i) {
        uint32_t w = col[i];
        if (w >= n) {
          bad = true;
          return;
        }
        if (w != v) b[d++] = w;
      }
      if (!std::is_sorted(b, b + d)) std::sort(b, b + d);
      keep[v] = (uint32_t)(std::unique(b, b + d) - b);
    }
  });
  if (bad) return kInvalidGraph;
  out.n = n;
  out.rp.assign((size_t)n + 1, 0);
  for (uint32_t v = 0; v < n; ++v) out.rp[v + 1] = out.rp[v] + keep[v];
  out.col.resize(out.rp[n]);
  parallel_chunks(n, 4096, threads, [&](uint64_t lo, uint64_t hi) {
    for (uint64_t v = lo; v < hi; ++v)
      std::memcpy(out.col.data() + out.rp[v], tmp.data() + rp[v], sizeof(uint32_t) * keep[v]);
  });
  return kOk;
}

void transpose(const Csr& g, Csr& t) {
  t.n = g.n;
  t.rp.assign((size_t)g.n + 1, 0);
  for (uint64_t i = 0; i < g.nnz(); ++i) ++t.rp[g.col[i] + 1];
  for (uint32_t v = 0; v < g.n; ++v) t.rp[v + 1] += t.rp[v];
  t.col.resize(g.nnz());
  std::vector<uint32_t> cur(t.rp.begin(), t.rp.end() - 1);
  for (uint32_t v = 0; v < g.n; ++v)  // rows visited in order: each in-list ends up sorted
    for (uint32_t i = g.rp[v]; i < g.rp[v + 1]; ++i) t.col[cur[g.col[i]]++] = v;
}

void undirected(const Csr& g, const Csr& gt, Csr& u) {
  u.n = g.n;
  u.rp.assign((size_t)g.n + 1, 0);
  std::vector<uint32_t> merged;
  std::vector<uint32_t> deg(g.n);
  for (uint32_t v = 0; v < g.n; ++v) {
    const uint32_t *a = g.col.data() + g.rp[v], *ae = g.col.data() + g.rp[v + 1];
    const uint32_t *b = gt.col.data() + gt.rp[v], *be = gt.col.data() + gt.rp[v + 1];
    uint32_t d = 0;
    while (a != ae || b != be) {
      if (b == be || (a != ae && *a < *b)) ++a;
      else if (a == ae || *b < *a) ++b;
      else { ++a; ++b; }
      ++d;
    }
    deg[v] = d;
  }
  for (uint32_t v = 0; v < g.n; ++v) u.rp[v + 1] = u.rp[v] + deg[v];
  u.col.resize(u.rp[g.n]);
  for (uint32_t v = 0; v < g.n; ++v) {
    uint32_t* o = u.col.data() + u.rp[v];
    std::set_union(g.col.data() + g.rp[v], g.col.data() + g.rp[v + 1], gt.col.data() + gt.rp[v],
                   gt.col.data() + gt.rp[v + 1], o);
  }
}

void relabel(const Csr& g, const std::vector<uint32_t>& new_id, int threads, Csr& out) {
  std::vector<uint32_t> inv(g.n);
  for (uint32_t v = 0; v < g.n; ++v) inv[new_id[v]] = v;
  out.n = g.n;
  out.rp.assign((size_t)g.n + 1, 0);
  for (uint32_t w = 0; w < g.n; ++w) out.rp[w + 1] = out.rp[w] + (g.rp[inv[w] + 1] - g.rp[inv[w]]);
  out.col.resize(g.nnz());
  parallel_chunks(g.n, 4096, threads, [&](uint64_t lo, uint64_t hi) {
    for (uint64_t w = lo; w < hi; ++w) {
      uint32_t v = inv[w];
      uint32_t* o = out.col.data() + out.rp[w];
      uint32_t d = g.rp[v + 1] - g.rp[v];
      for (uint32_t i = 0; i < d; ++i) o[i] = new_id[g.col[g.rp[v] + i]];
      std::sort(o, o + d);
    }
  });
}

// ---------------------------------------------------------------------------
// Social-like test (Section 2.2.1).  Heavy tail: the ceil(1%) and ceil(10%)
// highest-degree vertices hold more than 5% and more than 40% of the degree sum.
// Power law: the least-squares line through (log d, log count(d)) over degrees
// with a non-zero count (at least three) has slope in [-3.5, -1.5] and R^2 >= 0.9.
// ---------------------------------------------------------------------------
bool social_like(const Csr& g) {
  if (g.n == 0) return false;
  uint64_t total = g.nnz();
  if (total == 0) return false;
  uint32_t maxd = 0;
  for (uint32_t v = 0; v < g.n; ++v) maxd = std::max(maxd, g.rp[v + 1] - g.rp[v]);
  std::vector<uint64_t> hist((size_t)maxd + 1, 0);
  for (uint32_t v = 0; v < g.n; ++v) ++hist[g.rp[v + 1] - g.rp[v]];
  auto top_sum = [&](uint64_t count) {
    uint64_t s = 0;
    for (int64_t d = maxd; d >= 0 && count > 0; --d) {
      uint64_t take = std::min<uint64_t>(count, hist[d]);
      s += take * (uint64_t)d;
      count -= take;
    }
    return s;
  };
  uint64_t top1 = std::max<uint64_t>(1, (uint64_t)std::ceil(0.01 * (double)g.n));
  uint64_t top10 = std::max<uint64_t>(1, (uint64_t)std::ceil(0.10 * (double)g.n));
  bool heavy = (double)top_sum(top1) / (double)total > 0.05 && (double)top_sum(top10) / (double)total > 0.40;
  if (heavy) return true;
  std::vector<double> x, y;
  for (uint32_t d = 1; d <= maxd; ++d)
    if (hist[d]) {
      x.push_back(std::log((double)d));
      y.push_back(std::log((double)hist[d]));
    }
  if (x.size() < 3) return false;
  double xm = std::accumulate(x.begin(), x.end(), 0.0) / x.size();
  double ym = std::accumulate(y.begin(), y.end(), 0.0) / y.size();
  double sxx = 0, sxy = 0, syy = 0;
  for (size_t i = 0; i < x.size(); ++i) {
    sxx += (x[i] - xm) * (x[i] - xm);
    sxy += (x[i] - xm) * (y[i] - ym);
    syy += (y[i] - ym) * (y[i] - ym);
  }
  double slope = sxy / sxx;
  double res = 0;
  for (size_t i = 0; i < x.size(); ++i) {
    double e = y[i] - (ym + slope * (x[i] - xm));
    res += e * e;
  }
  double r2 = syy > 0 ? 1.0 - res / syy : 0.0;
  return slope >= -3.5 && slope <= -1.5 && r2 >= 0.9;
}

// ---------------------------------------------------------------------------
// Algorithm 1 (JaccardWithWindows).  Each window [s, e) is clustered
// independently: pop the smallest remaining vertex as the seed, then sigma - 1
// times take the remaining vertex j maximising |N(j) & U| / |N(j) | U| (ties: the
// smallest ID; all-zero scores: the smallest remaining ID) and grow U.
//
// Exact but fast: inter[j] = |N(j) & U| is kept incrementally through the
// in-neighbour lists of the vertices entering U (restricted to the window by a
// binary search), so only vertices sharing a neighbour with U are candidates; the
// argmax scans those candidates and compares scores i / (|N(j)| + |U| - i) by
// exact integer cross-multiplication.
// ---------------------------------------------------------------------------
void jaccard_windows(const Csr& g, const Csr& gt, uint32_t sigma, uint32_t w, int threads,
                     std::vector<uint32_t>& new_id) {
  const uint32_t n = g.n;
  new_id.assign(n, 0);
  const uint32_t nwin = (n + w - 1) / w;
  std::atomic<uint32_t> next_win(0);
  auto worker = [&] {
    std::vector<uint32_t> stamp(n, 0);
    uint32_t cid = 0;
    std::vector<uint8_t> rem;
    std::vector<uint32_t> inter, touched;
    for (;;) {
      uint32_t k = next_win.fetch_add(1);
      if (k >= nwin) return;
      const uint32_t s = k * w, e = (uint32_t)std::min<uint64_t>(n, (uint64_t)s + w);
      const uint32_t L = e - s;
      rem.assign(L, 1);
      inter.assign(L, 0);
      uint32_t remaining = L, pop_ptr = 0;
      uint64_t usize = 0;
      touched.clear();
      auto add_to_u = [&](uint32_t j) {
        for (uint32_t a = g.rp[j]; a < g.rp[j + 1]; ++a) {
          const uint32_t x = g.col[a];
          if (stamp[x] == cid) continue;
          stamp[x] = cid;
          ++usize;
          // in-neighbours of x inside the window gain x in N(j) & U
          const uint32_t* b = gt.col.data() + gt.rp[x];
          const uint32_t* be = gt.col.data() + gt.rp[x + 1];
          for (const uint32_t* p = std::lower_bound(b, be, s); p != be && *p < e; ++p) {
            const uint32_t li = *p - s;
            if (rem[li] && inter[li]++ == 0) touched.push_back(li);
          }
        }
      };
      const uint32_t M = (L + sigma - 1) / sigma;
      for (uint32_t ell = 0; ell < M; ++ell) {
        if (++cid == 0) {  // stamp wrap-around
          std::fill(stamp.begin(), stamp.end(), 0);
          cid = 1;
        }
        usize = 0;
        while (!rem[pop_ptr]) ++pop_ptr;
        const uint32_t jstar = s + pop_ptr;
        rem[pop_ptr] = 0;
        --remaining;
        new_id[jstar] = s + ell * sigma;
        add_to_u(jstar);
        for (uint32_t r = 1; r < sigma; ++r) {
          if (remaining == 0) break;
          uint64_t bi = 0, bd = 1;
          uint32_t bl = 0xFFFFFFFFu;  // best window-local index
          size_t out = 0;
          for (size_t t = 0; t < touched.size(); ++t) {
            const uint32_t li = touched[t];
            if (!rem[li]) continue;  // drop removed candidates while scanning
            touched[out++] = li;
            const uint64_t i = inter[li];
            const uint64_t d = (uint64_t)(g.rp[s + li + 1] - g.rp[s + li]) + usize - i;  // |N(j) | U|
            const unsigned __int128 lhs = (unsigned __int128)i * bd, rhs = (unsigned __int128)bi * d;
            if (lhs > rhs || (lhs == rhs && li < bl)) {
              bi = i;
              bd = d;
              bl = li;
            }
          }
          touched.resize(out);
          uint32_t jd;
          if (bl == 0xFFFFFFFFu) {  // every score is zero: smallest remaining ID
            while (!rem[pop_ptr]) ++pop_ptr;
            jd = s + pop_ptr;
          } else {
            jd = s + bl;
          }
          rem[jd - s] = 0;
          --remaining;
          new_id[jd] = s + ell * sigma + r;
          add_to_u(jd);
        }
        for (uint32_t li : touched) inter[li] = 0;
        touched.clear();
      }
    }
  };
  int T = std::min<int>(pick_threads(threads), (int)std::max<uint32_t>(1, nwin));
  std::vector<std::thread> th;
  for (int t = 1; t < T; ++t) th.emplace_back(worker);
  worker();
  for (auto& x : th) x.join();
}

// ---------------------------------------------------------------------------
// Reverse Cuthill-McKee on the undirected view.  Components in order of their
// smallest vertex; each is started from a George-Liu pseudo-peripheral vertex
// found from the component's minimum-(degree, ID) vertex, moving to the
// minimum-(degree, ID) vertex of the last BFS level while the eccentricity grows;
// neighbours are enqueued in (degree, ID) order; the whole order is reversed.
// ---------------------------------------------------------------------------
uint64_t splitmix64(uint64_t seed, uint64_t t) {
  uint64_t z = seed + t * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

void shingle_order(const Csr& g, uint32_t hashes, uint64_t seed, int threads, std::vector<uint32_t>& new_id) {
  const uint32_t n = g.n, k = hashes;
  std::vector<uint64_t> s(k);
  for (uint32_t i = 0; i < k; ++i) s[i] = splitmix64(seed, i + 1);
  // h_i(u) for every vertex, then each row's minimum per hash
  std::vector<uint64_t> h((size_t)n * k), key((size_t)n * k);
  parallel_chunks(n, 1 << 14, threads, [&](uint64_t lo, uint64_t hi) {
    for (uint64_t u = lo; u < hi; ++u)
      for (uint32_t i = 0; i < k; ++i) h[u * k + i] = splitmix64(s[i], u + 1);
  });
  parallel_chunks(n, 1 << 12, threads, [&](uint64_t lo, uint64_t hi) {
    for (uint64_t v = lo; v < hi; ++v) {
      uint64_t* kv = key.data() + v * k;
      for (uint32_t i = 0; i < k; ++i) kv[i] = ~0ull;
      for (uint32_t a = g.rp[v]; a < g.rp[v + 1]; ++a) {
        const uint64_t* hu = h.data() + (uint64_t)g.col[a] * k;
        for (uint32_t i = 0; i < k; ++i) kv[i] = std::min(kv[i], hu[i]);
      }
    }
  });
  std::vector<uint32_t> order(n);
  std::iota(order.begin(), order.end(), 0u);
  std::sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) {
    const uint64_t* ka = key.data() + (uint64_t)a * k;
    const uint64_t* kb = key.data() + (uint64_t)b * k;
    for (uint32_t i = 0; i < k; ++i)
      if (ka[i] != kb[i]) return ka[i] < kb[i];
    return a < b;
  });
  new_id.assign(n, 0);
  for (uint32_t r = 0; r < n; ++r) new_id[order[r]] = r;
}

void rcm(const Csr& u, std::vector<uint32_t>& new_id) {
  const uint32_t n = u.n;
  auto deg = [&](uint32_t v) { return u.rp[v + 1] - u.rp[v]; };
  auto better = [&](uint32_t a, uint32_t b) { return deg(a) < deg(b) || (deg(a) == deg(b) && a < b); };
  std::vector<uint8_t> seen(n, 0);
  std::vector<uint32_t> order;
  order.reserve(n);
  std::vector<int32_t> dist(n, -1);
  std::vector<uint32_t> comp, q;
  // BFS from root over the component; returns eccentricity and fills `last`.
  std::vector<uint32_t> last;
  auto ecc = [&](uint32_t root) {
    for (uint32_t v : comp) dist[v] = -1;
    q.clear();
    q.push_back(root);
    dist[root] = 0;
    int32_t maxd = 0;
    for (size_t h = 0; h < q.size(); ++h) {
      uint32_t v = q[h];
      for (uint32_t a = u.rp[v]; a < u.rp[v + 1]; ++a) {
        uint32_t w = u.col[a];
        if (dist[w] < 0) {
          dist[w] = dist[v] + 1;
          maxd = std::max(maxd, dist[w]);
          q.push_back(w);
        }
      }
    }
    last.clear();
    for (uint32_t v : q)
      if (dist[v] == maxd) last.push_back(v);
    return maxd;
  };
  std::vector<uint32_t> nb;
  for (uint32_t start = 0; start < n; ++start) {
    if (seen[start]) continue;
    comp.clear();
    comp.push_back(start);
    seen[start] = 2;  // 2 = collected into comp, not yet ordered
    for (size_t h = 0; h < comp.size(); ++h) {
      uint32_t v = comp[h];
      for (uint32_t a = u.rp[v]; a < u.rp[v + 1]; ++a)
        if (!seen[u.col[a]]) {
          seen[u.col[a]] = 2;
          comp.push_back(u.col[a]);
        }
    }
    uint32_t x = comp[0];
    for (uint32_t v : comp)
      if (better(v, x)) x = v;
    int32_t ex = ecc(x);
    for (;;) {
      uint32_t y = last[0];
      for (uint32_t v : last)
        if (better(v, y)) y = v;
      std::vector<uint32_t> saved_last = last;
      int32_t ey = ecc(y);
      if (ey > ex) {
        x = y;
        ex = ey;
      } else {
        last.swap(saved_last);
        break;
      }
    }
    // Cuthill-McKee from x
    size_t head = order.size();
    order.push_back(x);
    seen[x] = 1;
    for (; head < order.size(); ++head) {
      uint32_t v = order[head];
      nb.clear();
      for (uint32_t a = u.rp[v]; a < u.rp[v + 1]; ++a)
        if (seen[u.col[a]] != 1) nb.push_back(u.col[a]);
      std::sort(nb.begin(), nb.end(), better);
      for (uint32_t w : nb) {
        seen[w] = 1;
        order.push_back(w);
      }
    }
  }
  new_id.assign(n, 0);
  for (uint32_t i = 0; i < n; ++i) new_id[order[n - 1 - i]] = i;
}

// ---------------------------------------------------------------------------
// BVSS construction (Section 2.1).  Slice (u, i) exists iff u has an in-neighbour
// in columns [sigma*i, sigma*i + sigma); bit j of its mask is set iff the arc
// (sigma*i + j) -> u exists.  The slices of set i therefore come from merging the
// out-lists of vertices sigma*i .. sigma*i + sigma - 1.
// ---------------------------------------------------------------------------
int build_slices(const Csr& g, uint32_t sigma, uint32_t slots, int threads, Bvss& b) {
  b.n = g.n;
  b.sigma = sigma;
  b.slots = slots;
  b.tau = 64 * slots;
  b.num_sets = (g.n + sigma - 1) / sigma;
  const uint32_t S = b.num_sets;
  const uint32_t mb = sigma / 8;
  // Pass 1 and 2 per chunk of sets: merge into chunk-local buffers.
  const uint64_t chunk = 2048;
  const uint64_t nchunks = (S + chunk - 1) / chunk;
  std::vector<std::vector<uint32_t>> rows(nchunks);
  std::vector<std::vector<uint8_t>> masks(nchunks);
  std::vector<uint32_t> set_cnt(S, 0);
  parallel_chunks(nchunks, 1, threads, [&](uint64_t c0, uint64_t c1) {
    std::vector<uint64_t> keys;
    for (uint64_t c = c0; c < c1; ++c) {
      auto& R = rows[c];
      auto& Mk = masks[c];
      uint32_t s_lo = (uint32_t)(c * chunk), s_hi = (uint32_t)std::min<uint64_t>(S, (c + 1) * chunk);
      for (uint32_t s = s_lo; s < s_hi; ++s) {
        keys.clear();
        uint32_t v0 = s * sigma, v1 = std::min<uint32_t>(g.n, v0 + sigma);
        for (uint32_t v = v0; v < v1; ++v)
          for (uint32_t a = g.rp[v]; a < g.rp[v + 1]; ++a) keys.push_back(((uint64_t)g.col[a] << 6) | (v - v0));
        std::sort(keys.begin(), keys.end());
        uint32_t cnt = 0;
        for (size_t i = 0; i < keys.size();) {
          uint32_t row = (uint32_t)(keys[i] >> 6);
          uint64_t m = 0;
          for (; i < keys.size() && (uint32_t)(keys[i] >> 6) == row; ++i) m |= 1ull << (keys[i] & 63);
          R.push_back(row);
          for (uint32_t by = 0; by < mb; ++by) Mk.push_back((uint8_t)(m >> (8 * by)));
          ++cnt;
        }
        set_cnt[s] = cnt;
      }
    }
  });
  b.set_beg.assign((size_t)S + 1, 0);
  for (uint32_t s = 0; s < S; ++s) b.set_beg[s + 1] = b.set_beg[s] + set_cnt[s];
  b.num_slices = b.set_beg[S];
  b.row_ids.resize(b.num_slices);
  b.masks.resize(b.num_slices * mb);
  parallel_chunks(nchunks, 1, threads, [&](uint64_t c0, uint64_t c1) {
    for (uint64_t c = c0; c < c1; ++c) {
      uint64_t off = b.set_beg[c * chunk];
      std::memcpy(b.row_ids.data() + off, rows[c].data(), sizeof(uint32_t) * rows[c].size());
      std::memcpy(b.masks.data() + off * mb, masks[c].data(), masks[c].size());
      std::vector<uint32_t>().swap(rows[c]);
      std::vector<uint8_t>().swap(masks[c]);
    }
  });
  return kOk;
}

void partition_vss_into(const Bvss& b, uint32_t range_len, int threads, VssPartition& out) {
  const uint32_t S = b.num_sets;
  // VSS partition: cut each set's row-sorted slices into runs of at most tau that
  // also stay inside one row range of range_len IDs (no range split if 0).
  out.range_len = range_len;
  auto range_of = [&](uint32_t row) { return range_len ? row / range_len : 0u; };
  auto walk = [&](uint32_t s, auto&& emit) {
    uint32_t k = b.set_beg[s], e = b.set_beg[s + 1];
    while (k < e) {
      const uint32_t r = range_of(b.row_ids[k]);
      uint32_t j = k + 1;
      while (j < e && j - k < b.tau && range_of(b.row_ids[j]) == r) ++j;
      emit(k, r);
      k = j;
    }
  };
  std::vector<uint32_t> vss_cnt(S, 0);
  parallel_chunks(S, 4096, threads, [&](uint64_t lo, uint64_t hi) {
    for (uint64_t s = lo; s < hi; ++s) walk((uint32_t)s, [&](uint32_t, uint32_t) { ++vss_cnt[s]; });
  });
  out.real_ptrs.assign((size_t)S + 1, 0);
  for (uint32_t s = 0; s < S; ++s) out.real_ptrs[s + 1] = out.real_ptrs[s] + vss_cnt[s];
  out.num_vss = out.real_ptrs[S];
  out.v2r.resize(out.num_vss);
  out.vss_beg.resize((size_t)out.num_vss + 1);
  out.vss_range.resize(out.num_vss);
  parallel_chunks(S, 4096, threads, [&](uint64_t lo, uint64_t hi) {
    for (uint64_t s = lo; s < hi; ++s) {
      uint32_t v = out.real_ptrs[s];
      walk((uint32_t)s, [&](uint32_t k, uint32_t r) {
        out.v2r[v] = (uint32_t)s;
        out.vss_beg[v] = k;
        out.vss_range[v] = (uint8_t)r;
        ++v;
      });
    }
  });
  out.vss_beg[out.num_vss] = (uint32_t)b.num_slices;
}

int partition_vss(Bvss& b, uint32_t range_len, int threads) {
  VssPartition part;
  partition_vss_into(b, range_len, threads, part);
  b.range_len = part.range_len;
  b.num_vss = part.num_vss;
  b.real_ptrs = std::move(part.real_ptrs);
  b.v2r = std::move(part.v2r);
  b.vss_beg = std::move(part.vss_beg);
  b.vss_range = std::move(part.vss_range);
  return kOk;
}

double update_divergence(const Bvss& b, uint32_t lanes, uint32_t slots_per_lane) {
  const uint32_t tau = lanes * slots_per_lane;
  double sum = 0;
  uint64_t nvss = 0;
  auto vss = [&](uint32_t v, uint32_t ve) {
    double cols = 0;
    uint32_t ncols = 0;
    for (uint32_t c = v; c < ve; c += lanes) {
      uint32_t ce = std::min(ve, c + lanes);
      double mean = 0;
      for (uint32_t k = c; k < ce; ++k) mean += b.row_ids[k];
      mean /= (ce - c);
      double var = 0;
      for (uint32_t k = c; k < ce; ++k) var += (b.row_ids[k] - mean) * (b.row_ids[k] - mean);
      cols += std::sqrt(var / (ce - c));
      ++ncols;
    }
    sum += cols / ncols;
    ++nvss;
  };
  if (slots_per_lane == 0) {  // this layout's own VSSs, `lanes` per column
    for (uint32_t v = 0; v < b.num_vss; ++v) vss(b.vss_beg[v], b.vss_beg[v + 1]);
  } else {  // each set cut into VSSs of tau slices
    for (uint32_t s = 0; s < b.num_sets; ++s) {
      uint32_t lo = b.set_beg[s], hi = b.set_beg[s + 1];
      for (uint32_t v = lo; v < hi; v += tau) vss(v, std::min(hi, v + tau));
    }
  }
  return nvss ? sum / nvss : 0.0;
}

// Hub sort: sigma-aligned vertex groups (the future slice sets) are ranked by the
// summed in-degree of their members, largest first, ties kept in order; members
// keep their order inside a group.  Only groups inside complete 32-vertex words
// move (the tail stays in place), so slice sets and masks are unchanged, and so is
// the compression ratio.  Ranked groups fill words in rank order (32 / sigma
// groups per word), and ranked words go first to the cached positions of the
// lazy kernel's LDS cache - positions 0 .. cpos-1 of every 64-word chunk; the
// t-th round over the chunks gives chunk c position (t + c) mod cpos - then to the
// remaining positions in ascending order.  The hottest rows thus sit in the cache and are spread over all
// chunks, so that no single wavefront of the frontier sweep owns all hub sets.
void hub_sort(const Csr& g, uint32_t sigma, uint32_t cpos, std::vector<uint32_t>& new_id) {
  const uint32_t n = g.n;
  const uint32_t spw = 32 / sigma;          // groups per word
  const uint32_t fw = n / 32;               // complete words
  const uint64_t fg = (uint64_t)fw * spw;   // groups that move
  std::vector<uint64_t> w(fg, 0);
  for (uint64_t k = 0; k < g.nnz(); ++k) {
    const uint32_t grp = g.col[k] / sigma;
    if (grp < fg) w[grp] += 1;
  }
  std::vector<uint32_t> order(fg);
  for (uint32_t x = 0; x < fg; ++x) order[x] = x;
  std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) { return w[a] > w[b]; });
  std::vector<uint32_t> slot;
  slot.reserve(fw);
  std::vector<uint8_t> taken(fw, 0);
  const uint32_t chunks = (fw + 63) / 64;
  const uint32_t cp = std::min<uint32_t>(cpos, 64);
  for (uint32_t t = 0; t < cp; ++t)
    for (uint32_t c = 0; c < chunks; ++c) {
      // the position rotates with the chunk, so that equally hot words of
      // different chunks fall into different LDS banks
      const uint32_t q = c * 64 + (t + c) % cp;
      if (q < fw) {
        slot.push_back(q);
        taken[q] = 1;
      }
    }
  for (uint32_t q = 0; q < fw; ++q)
    if (!taken[q]) slot.push_back(q);
  new_id.resize(n);
  for (uint64_t r = 0; r < fg; ++r) {
    const uint64_t gnew = (uint64_t)slot[r / spw] * spw + r % spw;
    for (uint32_t j = 0; j < sigma; ++j) new_id[(uint64_t)order[r] * sigma + j] = (uint32_t)(gnew * sigma + j);
  }
  for (uint64_t v = fg * sigma; v < n; ++v) new_id[v] = (uint32_t)v;
}

}  // namespace blest
