// mstx_cpu.cpp -- the paper's CPU variants of Boruvka (Sections 2.1, 2.2.1,
// 2.2.2) as host code, for context beside the GPU library.  Interface and
// semantics: include/mstx_cpu.h.
//
// Edges are ordered by the key (w[e], e) everywhere (the paper assumes
// distinct weights; the index makes the order total), so every variant
// returns the same unique tree.  All memory that threads share is accessed
// through std::atomic; the phases of a round are separated by barriers, so a
// thread sanitizer reports nothing.

#include <algorithm>
#include <atomic>
#include <barrier>
#include <cstring>
#include <thread>
#include <vector>

#include "mstx_cpu.h"

namespace {

constexpr int64_t kNone = -1;

struct Graph {
  int32_t n;
  int64_t m;
  const int32_t* src;
  const int32_t* dst;
  const uint32_t* w;
  uint64_t key(int64_t e) const { return ((uint64_t)w[e] << 32) | (uint64_t)(uint32_t)e; }
  // whether edge e is lighter than the current minimum `cur` (kNone: no minimum yet)
  bool lighter(int64_t e, int64_t cur) const { return cur == kNone || key(e) < key(cur); }
};

int finish(const Graph& g, int64_t added, const std::vector<int64_t>& tree, uint8_t* in_mst, uint64_t* total) {
  std::memset(in_mst, 0, (size_t)g.m);
  uint64_t t = 0;
  for (int64_t e : tree) {
    if (in_mst[e]) return MSTX_ERR_DEVICE;  // an edge added twice: never expected
    in_mst[e] = 1;
    t += g.w[e];
  }
  *total = t;
  return (g.n <= 1 || added == (int64_t)g.n - 1) ? MSTX_OK : MSTX_DISCONNECTED;
}

// ------------------------------------------------------------- sequential

int32_t find_seq(std::vector<int32_t>& parent, int32_t x) {
  while (parent[x] != x) {
    parent[x] = parent[parent[x]];  // path halving
    x = parent[x];
  }
  return x;
}

// Section 2.1; `covered` enables the covered-edge optimisation.
int solve_sequential(const Graph& g, bool covered, uint8_t* in_mst, uint64_t* total, int64_t* rounds) {
  std::vector<int32_t> parent(g.n), size(g.n, 1);
  for (int32_t v = 0; v < g.n; ++v) parent[v] = v;
  std::vector<int64_t> minimum(g.n);
  std::vector<uint8_t> cov(covered ? g.m : 0, 0);
  std::vector<int64_t> tree;
  int64_t comps = g.n, r = 0;
  while (comps > 1) {
    std::fill(minimum.begin(), minimum.end(), kNone);
    bool any = false;
    for (int64_t e = 0; e < g.m; ++e) {
      if (covered && cov[e]) continue;
      const int32_t c1 = find_seq(parent, g.src[e]);
      const int32_t c2 = find_seq(parent, g.dst[e]);
      if (c1 == c2) {
        if (covered) cov[e] = 1;
        continue;
      }
      if (g.lighter(e, minimum[c1])) minimum[c1] = e;
      if (g.lighter(e, minimum[c2])) minimum[c2] = e;
      any = true;
    }
    if (!any) break;  // no component has an outgoing edge: a forest
    ++r;
    for (int32_t v = 0; v < g.n; ++v) {
      const int64_t e = minimum[v];
      if (e == kNone) continue;
      int32_t c1 = find_seq(parent, g.src[e]);
      int32_t c2 = find_seq(parent, g.dst[e]);
      if (c1 == c2) continue;  // the partner component added it already
      tree.push_back(e);
      if (covered) cov[e] = 1;
      if (size[c1] < size[c2]) std::swap(c1, c2);  // the bigger component keeps its root
      parent[c2] = c1;
      size[c1] += size[c2];
      --comps;
    }
  }
  if (rounds) *rounds = r;
  return finish(g, (int64_t)tree.size(), tree, in_mst, total);
}

// --------------------------------------------------------------- parallel

struct Parallel {
  const Graph& g;
  const int T;
  const bool locks;  // Section 2.2.1 (permission words) or 2.2.2 (CAS)
  std::vector<std::atomic<int32_t>> parent, owner, perm;
  std::vector<std::atomic<uint8_t>> covered;
  std::vector<int64_t> minimum;  // minimum[c] is written only by owner(c) in the scan phase
  std::vector<std::vector<int64_t>> tree;  // per thread
  std::atomic<int64_t> found[2], added[2];
  std::barrier<> bar;
  int64_t rounds = 0;

  Parallel(const Graph& gr, int threads, bool use_locks)
      : g(gr), T(threads), locks(use_locks), parent(gr.n), owner(gr.n), perm(use_locks ? gr.n : 0),
        covered(gr.m), minimum(gr.n, kNone), tree(threads), bar(threads) {
    for (int32_t v = 0; v < g.n; ++v) {
      parent[v].store(v, std::memory_order_relaxed);
      // contiguous blocks of vertices per thread
      owner[v].store((int32_t)((int64_t)v * T / std::max<int32_t>(g.n, 1)), std::memory_order_relaxed);
      if (locks) perm[v].store(-1, std::memory_order_relaxed);
    }
    for (int64_t e = 0; e < g.m; ++e) covered[e].store(0, std::memory_order_relaxed);
    for (int i = 0; i < 2; ++i) {
      found[i].store(0);
      added[i].store(0);
    }
  }

  // Root of x; path halving stores only into non-roots, and only ancestors.
  int32_t find(int32_t x) {
    for (;;) {
      const int32_t p = parent[x].load(std::memory_order_relaxed);
      if (p == x) return x;
      const int32_t gp = parent[p].load(std::memory_order_relaxed);
      if (gp == p) return p;
      parent[x].store(gp, std::memory_order_relaxed);
      x = gp;
    }
  }

  bool try_take(int32_t c, int tid) {
    int32_t expect = -1;
    return perm[c].compare_exchange_strong(expect, tid, std::memory_order_acq_rel);
  }
  void give_back(int32_t c) { perm[c].store(-1, std::memory_order_release); }

  // Unites the two components that minimum[v]'s edge joins; true if the edge
  // was added.
  bool unite(int64_t e, int tid) {
    const int32_t c1 = find(g.src[e]);
    const int32_t c2 = find(g.dst[e]);
    if (c1 == c2) {
      covered[e].store(1, std::memory_order_relaxed);
      return false;
    }
    // The larger root goes under the smaller one.  Parent pointers then
    // always decrease, so no cycle can form even though the two finds above
    // ran at different moments (c1 may have been linked since): a root can
    // never be linked under one of its own descendants.
    const int32_t lo = std::min(c1, c2), hi = std::max(c1, c2);
    if (!locks) {
      // one compare-and-swap: hi's root pointer from itself to lo
      int32_t expect = hi;
      if (!parent[hi].compare_exchange_strong(expect, lo, std::memory_order_acq_rel)) return false;
    } else {
      // permission on both components (lower id first), no spinning
      if (!try_take(lo, tid)) return false;
      if (!try_take(hi, tid)) {
        give_back(lo);
        return false;
      }
      // with both permissions held nobody else can change either root
      const bool roots = parent[lo].load(std::memory_order_acquire) == lo &&
                         parent[hi].load(std::memory_order_acquire) == hi;
      if (roots) parent[hi].store(lo, std::memory_order_release);
      give_back(hi);
      give_back(lo);
      if (!roots) return false;
    }
    owner[lo].store(tid, std::memory_order_relaxed);
    covered[e].store(1, std::memory_order_relaxed);
    tree[tid].push_back(e);
    return true;
  }

  void run(int tid) {
    for (int64_t r = 0;; ++r) {
      const int cur = (int)(r & 1), nxt = cur ^ 1;
      for (int32_t v = 0; v < g.n; ++v)
        if (owner[v].load(std::memory_order_relaxed) == tid) minimum[v] = kNone;
      bar.arrive_and_wait();
      if (tid == 0) {
        // the other parity's counters were last read before the previous barrier
        found[nxt].store(0);
        added[nxt].store(0);
      }
      // every thread walks all edges, starting at its own evenly spaced edge
      int64_t mine = 0;
      const int64_t start = g.m * tid / T;
      for (int64_t i = 0; i < g.m; ++i) {
        int64_t e = start + i;
        if (e >= g.m) e -= g.m;
        if (covered[e].load(std::memory_order_relaxed)) continue;
        const int32_t c1 = find(g.src[e]);
        const int32_t c2 = find(g.dst[e]);
        if (c1 == c2) {
          covered[e].store(1, std::memory_order_relaxed);
          continue;
        }
        if (owner[c1].load(std::memory_order_relaxed) == tid && g.lighter(e, minimum[c1])) {
          minimum[c1] = e;
          ++mine;
        }
        if (owner[c2].load(std::memory_order_relaxed) == tid && g.lighter(e, minimum[c2])) {
          minimum[c2] = e;
          ++mine;
        }
      }
      found[cur].fetch_add(mine);
      bar.arrive_and_wait();
      if (found[cur].load() == 0) {
        if (tid == 0) rounds = r;
        return;  // no component has an outgoing edge
      }
      int64_t done = 0;
      for (int32_t v = 0; v < g.n; ++v) {
        if (owner[v].load(std::memory_order_relaxed) != tid) continue;
        if (parent[v].load(std::memory_order_relaxed) != v || minimum[v] == kNone) continue;
        done += unite(minimum[v], tid) ? 1 : 0;
      }
      added[cur].fetch_add(done);
      bar.arrive_and_wait();
      if (added[cur].load() == 0) {
        // every permission attempt of the round failed: one thread unites
        // alone, so each round makes progress
        if (tid == 0)
          for (int32_t v = 0; v < g.n; ++v)
            if (parent[v].load(std::memory_order_relaxed) == v && minimum[v] != kNone) unite(minimum[v], 0);
        bar.arrive_and_wait();
      }
    }
  }
};

int solve_parallel(const Graph& g, int threads, bool locks, uint8_t* in_mst, uint64_t* total, int64_t* rounds) {
  Parallel P(g, threads, locks);
  std::vector<std::thread> pool;
  for (int t = 1; t < threads; ++t) pool.emplace_back([&P, t] { P.run(t); });
  P.run(0);
  for (auto& th : pool) th.join();
  std::vector<int64_t> all;
  for (auto& v : P.tree) all.insert(all.end(), v.begin(), v.end());
  if (rounds) *rounds = P.rounds;
  return finish(g, (int64_t)all.size(), all, in_mst, total);
}

}  // namespace

extern "C" {

int mst_cpu_solve(int variant, int32_t threads, int32_t n, int64_t m, const int32_t* src, const int32_t* dst,
                  const uint32_t* w, uint8_t* out_in_mst, uint64_t* out_total, int64_t* out_rounds) {
  if (variant < MSTX_CPU_SEQ_PLAIN || variant > MSTX_CPU_PAR_CAS) return MSTX_ERR_INVALID_ARG;
  if (n < 0 || m < 0 || !out_total) return MSTX_ERR_INVALID_ARG;
  if (m > (int64_t)0xFFFFFFFFLL) return MSTX_ERR_TOO_LARGE;
  if (m > 0 && (!src || !dst || !w || !out_in_mst)) return MSTX_ERR_INVALID_ARG;
  if (variant >= MSTX_CPU_PAR_LOCK && (threads < 1 || threads > 1024)) return MSTX_ERR_INVALID_ARG;
  for (int64_t e = 0; e < m; ++e)
    if ((uint32_t)src[e] >= (uint32_t)n || (uint32_t)dst[e] >= (uint32_t)n) return MSTX_ERR_VERTEX_RANGE;
  const Graph g{n, m, src, dst, w};
  if (out_rounds) *out_rounds = 0;
  if (m == 0) {
    *out_total = 0;
    return n <= 1 ? MSTX_OK : MSTX_DISCONNECTED;
  }
  switch (variant) {
    case MSTX_CPU_SEQ_PLAIN: return solve_sequential(g, false, out_in_mst, out_total, out_rounds);
    case MSTX_CPU_SEQ_COVERED: return solve_sequential(g, true, out_in_mst, out_total, out_rounds);
    case MSTX_CPU_PAR_LOCK: return solve_parallel(g, threads, true, out_in_mst, out_total, out_rounds);
    default: return solve_parallel(g, threads, false, out_in_mst, out_total, out_rounds);
  }
}

const char* mst_cpu_variant_name(int variant) {
  switch (variant) {
    case MSTX_CPU_SEQ_PLAIN: return "sequential";
    case MSTX_CPU_SEQ_COVERED: return "sequential_covered";
    case MSTX_CPU_PAR_LOCK: return "parallel_lock";
    case MSTX_CPU_PAR_CAS: return "parallel_cas";
    default: return "";
  }
}

}  // extern "C"
