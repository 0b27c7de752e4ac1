/*
 * Oracle: plain breadth-first search on the CPU.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this file's library.  It shares no code,
 * header or table with the GPU library, which must never call it.
 *
 * What it computes is the plain definition of the BFS output in the paper's
 * problem statement (Section 2, "Background and Notation"): level[u] is the length
 * of a shortest source-to-u path along out-edges, and parent[u] is the previous
 * vertex on one such path.  It is a first-in-first-out queue BFS, one vertex at a
 * time, with no blocking, bitmaps or reordering.  Unreached vertices get -1 (the
 * paper's infinity).  The pull formulation of the method (y = A (x) x over the
 * Boolean semiring, with A the adjacency of the transposed graph) reaches exactly
 * the same levels, which is what the GPU path is checked against.
 *
 * The graph is a CSR of out-neighbours with 32-bit offsets (n + 1 entries) and
 * 32-bit column indices.
 */
#include <stdint.h>
#include <stdlib.h>

/* Single-source BFS.  level[n] receives the hop count (-1 if unreachable).
 * parent may be NULL; otherwise parent[source] = source, parent[v] = the vertex
 * whose dequeue discovered v, and -1 for unreached vertices.
 * Returns 0, or -1 if source >= n or memory runs out. */
int oracle_bfs(uint32_t n, const uint32_t* row_ptr, const uint32_t* col, uint32_t source,
               int32_t* level, int32_t* parent) {
  if (source >= n) return -1;
  uint32_t* queue = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)n);
  if (!queue) return -1;
  for (uint32_t v = 0; v < n; ++v) {
    level[v] = -1;
    if (parent) parent[v] = -1;
  }
  uint32_t head = 0, tail = 0;
  level[source] = 0;
  if (parent) parent[source] = (int32_t)source;
  queue[tail++] = source;
  while (head < tail) {
    uint32_t v = queue[head++];
    for (uint32_t i = row_ptr[v]; i < row_ptr[v + 1]; ++i) {
      uint32_t w = col[i];
      if (level[w] == -1) {
        level[w] = level[v] + 1;
        if (parent) parent[w] = (int32_t)v;
        queue[tail++] = w;
      }
    }
  }
  free(queue);
  return 0;
}

/* k independent BFSs; row j of levels (levels[j*n .. j*n+n-1]) belongs to
 * sources[j].  Returns 0, or the negative status of the first failing row. */
int oracle_bfs_multi(uint32_t n, const uint32_t* row_ptr, const uint32_t* col, const uint32_t* sources,
                     uint32_t k, int32_t* levels) {
  for (uint32_t j = 0; j < k; ++j) {
    int rc = oracle_bfs(n, row_ptr, col, sources[j], levels + (size_t)j * n, NULL);
    if (rc != 0) return rc;
  }
  return 0;
}

static int has_arc(const uint32_t* row_ptr, const uint32_t* col, uint32_t u, uint32_t v) {
  /* neighbour lists are sorted: binary search */
  uint32_t lo = row_ptr[u], hi = row_ptr[u + 1];
  while (lo < hi) {
    uint32_t mid = lo + (hi - lo) / 2;
    if (col[mid] < v) lo = mid + 1;
    else hi = mid;
  }
  return lo < row_ptr[u + 1] && col[lo] == v;
}

/* Graph500-style check of a BFS tree against a level array that is known to be
 * right (the oracle's).  Returns 0 if valid, otherwise the number of the first
 * rule that fails:
 *   1  parent[source] != source
 *   2  a reached v != source whose parent p has no arc p -> v
 *   3  level[parent[v]] != level[v] - 1
 *   4  parent[v] set exactly for reached vertices (parent[v] == -1 iff level[v] == -1)
 *   5  an arc u -> v with u reached and (v unreached or level[v] > level[u] + 1)
 *   6  a parent index out of range
 */
int oracle_validate_tree(uint32_t n, const uint32_t* row_ptr, const uint32_t* col, uint32_t source,
                         const int32_t* level, const int32_t* parent) {
  if (source >= n || parent[source] != (int32_t)source) return 1;
  for (uint32_t v = 0; v < n; ++v) {
    if ((parent[v] == -1) != (level[v] == -1)) return 4;
    if (level[v] == -1 || v == source) continue;
    if (parent[v] < 0 || (uint32_t)parent[v] >= n) return 6;
    uint32_t p = (uint32_t)parent[v];
    if (!has_arc(row_ptr, col, p, v)) return 2;
    if (level[p] != level[v] - 1) return 3;
  }
  for (uint32_t u = 0; u < n; ++u) {
    if (level[u] == -1) continue;
    for (uint32_t i = row_ptr[u]; i < row_ptr[u + 1]; ++i) {
      uint32_t v = col[i];
      if (level[v] == -1 || level[v] > level[u] + 1) return 5;
    }
  }
  return 0;
}
