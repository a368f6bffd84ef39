// mstx_batched.hip -- kernels of the batched solve (many independent graphs in one call).
//
// The minimum spanning forest of a disjoint union of graphs is the union of
// their forests, and Boruvka never merges components of different graphs, so
// a batch is solved in four parts:
//
//   * graphs with at most kSmallN vertices whose edges fit in LDS behind the
//     vertex state: one workgroup per graph runs every Boruvka round of
//     Section 2.1 with the vertex state (component of each vertex, union-find
//     parents, minimum keys) and the edges in LDS; rounds are separated by
//     workgroup barriers only, so thousands of small graphs proceed
//     independently and in parallel;
//   * the other graphs with up to kMidN vertices and kMidMaxEdges edges: one
//     workgroup per graph as well, 10 bytes of LDS per vertex (minimum key and
//     a 2-byte union-find), the edges streamed from memory every round and a
//     dense finish on a pair table (the mid-size solve);
//   * graphs with up to kPreMaxN vertices (same edge bound): one workgroup per
//     graph contracts it round by round until at most kMidN components are
//     left, then the mid-size solve finishes the contracted graph;
//   * larger graphs: gathered into chunks that are solved as one disjoint
//     union by the single-graph round kernels (k_gather renumbers vertices and
//     edges into the union, k_graph_epilogue scatters the flags back and sums
//     per graph).
//
// Edge keys are (w << 32) | local edge index, so ties break by position inside
// the graph as in the single-graph solve.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <stdint.h>

#include "mstx.h"
#include "mstx_internal.h"

namespace mstx {

static constexpr int kSmallBlock = 1024;

__device__ __forceinline__ int32_t lds_load(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Root of x in the LDS union-find `par` (parents always point to smaller ids).
__device__ __forceinline__ int32_t small_root(int32_t* par, int32_t x) {
  int32_t p = lds_load(par + x);
  while (p != x) {
    const int32_t gp = lds_load(par + p);
    if (gp == p) return p;
    par[x] = gp;  // halving: gp is an ancestor of x
    x = gp;
    p = lds_load(par + x);
  }
  return x;
}

__device__ __forceinline__ uint32_t small_wave_sum(uint32_t v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// One workgroup per graph of `glist` (graphs with n <= kSmallN).  LDS holds
// best[n] (u64 minimum key per component root), comp[n] (round-start root of
// each vertex) and par[n] (union-find over the roots during hooking), and the
// graph's edges when they fit behind them.  Each round: minima over the
// graph's edges (from LDS, else re-read from HBM / cache), CAS hooking
// of the larger root under the smaller, compression; the loop ends when a
// round selects no edge.  Writes in_mst for the graph's edges (zeroed by the
// caller), total[g] and status[g].
//
// With glist == nullptr the launch is one workgroup for the single graph
// (n_single, m_single), and `stats` (when not null) receives the round
// statistics in the single-graph form: stats[0] = rows, then per row
// (components entering the round, isolated ones dropped; edges between
// different components; edges added).
// (The body of one workgroup, item `item` of glist; sbest is the dynamic LDS.)
// sbest: [n] minima, then comp [n], par [n], the edge cache
__device__ __forceinline__ void small_solve_body(unsigned long long* sbest, int item, const int32_t* __restrict__ glist,
                                                 const int64_t* __restrict__ voff, const int64_t* __restrict__ eoff,
                                                 int32_t n_single, int64_t m_single, const int32_t* __restrict__ src,
                                                 const int32_t* __restrict__ dst, const uint32_t* __restrict__ w,
                                                 uint8_t* __restrict__ in_mst,
                                                 unsigned long long* __restrict__ total_out,
                                                 int32_t* __restrict__ status_out, int64_t* __restrict__ stats,
                                                 uint32_t lds_bytes) {
  __shared__ uint32_t round_sel;
  __shared__ uint32_t bad;
  __shared__ unsigned long long red_w[kSmallBlock / 64];
  __shared__ uint32_t red_c[kSmallBlock / 64];
  __shared__ uint32_t round_live, round_nonisolated;

  const int g = glist ? glist[item] : 0;
  const int64_t e0 = glist ? eoff[g] : 0;
  const int64_t m = glist ? eoff[g + 1] - e0 : m_single;
  const int32_t n = glist ? (int32_t)(voff[g + 1] - voff[g]) : n_single;
  const int tid = threadIdx.x;
  int64_t n_round = n;  // components entering the round (statistics)
  int rows = 0;
  int32_t* comp = reinterpret_cast<int32_t*>(sbest + n);
  int32_t* par = comp + n;
  // The graph's edges stay in LDS behind the vertex state when they fit
  // (12 B each): every round then reads them from LDS instead of HBM / L2.
  const uint64_t cache_at = ((uint64_t)16 * (uint32_t)n + 15) & ~(uint64_t)15;
  const bool cached = cache_at + 12 * (uint64_t)m <= lds_bytes;
  int32_t* csrc = reinterpret_cast<int32_t*>(reinterpret_cast<char*>(sbest) + cache_at);
  int32_t* cdst = csrc + m;
  uint32_t* cw = reinterpret_cast<uint32_t*>(cdst + m);
  if (cached) {
    // eight edges per thread in flight at a time (loads clamped to edge 0,
    // the graph has one when m > 0, then stored for the edges that exist)
    for (int64_t j0 = 0; j0 < m; j0 += 8 * kSmallBlock) {
      int32_t a[8], b[8];
      uint32_t c[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int64_t j = j0 + q * kSmallBlock + tid;
        const int64_t jc = j < m ? j : 0;
        a[q] = src[e0 + jc];
        b[q] = dst[e0 + jc];
        c[q] = w[e0 + jc];
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int64_t j = j0 + q * kSmallBlock + tid;
        if (j < m) {
          csrc[j] = a[q];
          cdst[j] = b[q];
          cw[j] = c[q];
        }
      }
    }
  }
  const int32_t* esrc = cached ? csrc : src + e0;
  const int32_t* edst = cached ? cdst : dst + e0;
  const uint32_t* ew = cached ? cw : w + e0;

  for (int32_t v = tid; v < n; v += kSmallBlock) comp[v] = v;
  if (tid == 0) bad = 0;
  unsigned long long my_w = 0;
  uint32_t my_cnt = 0;
  __syncthreads();

  for (int round = 0; round < kMaxRounds; ++round) {
    for (int32_t v = tid; v < n; v += kSmallBlock) {
      sbest[v] = kKeyNone;
      par[v] = v;
    }
    if (tid == 0) {
      round_sel = 0;
      round_live = 0;
      round_nonisolated = 0;
    }
    __syncthreads();
    // edge scan: lightest outgoing key per component root
    uint32_t live = 0;
    for (int64_t j = tid; j < m; j += kSmallBlock) {
      const int32_t a0 = esrc[j], b0 = edst[j];
      if ((uint32_t)a0 >= (uint32_t)n || (uint32_t)b0 >= (uint32_t)n) {
        bad = 1;
        continue;
      }
      const int32_t a = comp[a0], b = comp[b0];
      if (a == b) continue;
      ++live;
      const unsigned long long key = ((unsigned long long)ew[j] << 32) | (unsigned long long)j;
      if (key < sbest[a]) atomicMin(sbest + a, key);
      if (key < sbest[b]) atomicMin(sbest + b, key);
    }
    // round counters: one LDS atomic per wave (1024 same-address atomics
    // would serialise)
    if (stats) {
      live = small_wave_sum(live);
      if ((tid & 63) == 0 && live) atomicAdd(&round_live, live);
    }
    __syncthreads();
    // hooking: every root with a minimum unites with the other end's root
    uint32_t sel = 0, nonisolated = 0;
    for (int32_t c = tid; c < n; c += kSmallBlock) {
      if (comp[c] != c) continue;
      const unsigned long long key = sbest[c];
      if (key == kKeyNone) continue;
      ++nonisolated;
      const int64_t j = (int64_t)(uint32_t)key;
      const int32_t u = comp[esrc[j]], v = comp[edst[j]];
      const int32_t d = (u == c) ? v : u;
      if (d < c && sbest[d] == key) continue;  // mutual choice: d hooks it
      int32_t x = c, y = d;
      while (true) {
        const int32_t rx = small_root(par, x);
        const int32_t ry = small_root(par, y);
        if (rx == ry) break;
        const int32_t hi = rx > ry ? rx : ry;
        const int32_t lo = rx > ry ? ry : rx;
        const int32_t old = atomicCAS(par + hi, hi, lo);
        if (old == hi) {
          in_mst[e0 + j] = 1;
          my_w += (uint32_t)(key >> 32);
          ++sel;
          break;
        }
        if (hi == rx) x = old;
        else y = old;
      }
    }
    my_cnt += sel;
    sel = small_wave_sum(sel);
    if ((tid & 63) == 0 && sel) atomicAdd(&round_sel, sel);
    nonisolated = small_wave_sum(nonisolated);
    if ((tid & 63) == 0 && nonisolated) atomicAdd(&round_nonisolated, nonisolated);
    __syncthreads();
    if (stats && tid == 0 && (round == 0 || n_round > 1) && !bad) {
      // a row for every round the single-graph path would run
      stats[1 + 3 * rows + 0] = n_round;
      stats[1 + 3 * rows + 1] = round_live;
      stats[1 + 3 * rows + 2] = round_sel;
    }
    if (round == 0 || n_round > 1) ++rows;
    // isolated components (no outgoing edge) leave; each added edge merges two
    n_round = (int64_t)round_nonisolated - (int64_t)round_sel;
    // done when no edge was added, or when at most one component with an
    // outgoing edge is left (its edges can only lead to itself: a component
    // without one never gains one)
    if (round_sel == 0 || n_round <= 1) break;
    // compression: the final root of every root of this round goes to a buffer
    // of its own (the minima are no longer needed), so a concurrent halving
    // store into par[] cannot replace it; then every vertex takes its root's root
    int32_t* newroot = reinterpret_cast<int32_t*>(sbest);
    for (int32_t c = tid; c < n; c += kSmallBlock) {
      if (comp[c] == c) newroot[c] = small_root(par, c);
    }
    __syncthreads();
    for (int32_t v = tid; v < n; v += kSmallBlock) comp[v] = newroot[comp[v]];
    __syncthreads();
  }
  // per-graph totals
  for (int off = 32; off > 0; off >>= 1) {
    my_w += __shfl_xor(my_w, off, 64);
    my_cnt += __shfl_xor(my_cnt, off, 64);
  }
  if ((tid & 63) == 0) {
    red_w[tid >> 6] = my_w;
    red_c[tid >> 6] = my_cnt;
  }
  __syncthreads();
  if (tid == 0) {
    unsigned long long tw = 0;
    uint32_t tc = 0;
    for (int i = 0; i < kSmallBlock / 64; ++i) {
      tw += red_w[i];
      tc += red_c[i];
    }
    total_out[g] = tw;
    int32_t st = (n <= 1 || (int64_t)tc == (int64_t)n - 1) ? MSTX_OK : MSTX_DISCONNECTED;
    if (bad) st = MSTX_ERR_VERTEX_RANGE;
    status_out[g] = st;
    if (stats) stats[0] = rows;
  }
}

__global__ void __launch_bounds__(kSmallBlock) k_small_solve(const int32_t* __restrict__ glist,
                                                             const int64_t* __restrict__ voff,
                                                             const int64_t* __restrict__ eoff,
                                                             int32_t n_single, int64_t m_single,
                                                             const int32_t* __restrict__ src,
                                                             const int32_t* __restrict__ dst,
                                                             const uint32_t* __restrict__ w,
                                                             uint8_t* __restrict__ in_mst,
                                                             unsigned long long* __restrict__ total_out,
                                                             int32_t* __restrict__ status_out,
                                                             int64_t* __restrict__ stats, uint32_t lds_bytes) {
  extern __shared__ unsigned long long dyn_lds[];
  small_solve_body(dyn_lds, blockIdx.x, glist, voff, eoff, n_single, m_single, src, dst, w, in_mst, total_out,
                   status_out, stats, lds_bytes);
}

// ---------------------------------------------------------------- mid-size

static constexpr int kMidBlock = 1024;
static constexpr int kMidUnroll = 8;      // edges per thread with loads in flight
static constexpr int kMidPerThread = 16;  // vertices per thread (registers)
static_assert(kMidN <= kMidPerThread * kMidBlock, "every vertex has a register slot");
static_assert(kMidN < 65536, "vertex ids fit the 2-byte union-find");
// The mid-size solve's dense finish: at most kMidDense components with an
// outgoing edge left.  LDS then holds a byte per vertex twice (root numbers,
// vertex numbers), the minimum key of every component pair, and the minima,
// parents and round-start roots of the components.
static constexpr int32_t kMidDense = 178;
__host__ __device__ constexpr size_t mid_dense_pairs_at(int32_t n) { return ((size_t)2 * (size_t)n + 7) & ~(size_t)7; }
static_assert(mid_dense_pairs_at(kMidN) + 8 * (size_t)kMidDense * (kMidDense - 1) / 2 + 16 * (size_t)kMidDense <=
                  (size_t)kMaxDynLds,
              "the dense finish fits the LDS allocation");
static_assert(kMidDense < 255 && kMidDense <= kMidBlock, "dense numbers fit a byte; one thread per component");

// The union-find of a mid-size graph: one u16 per vertex in LDS.  At the
// start of a round it is flat (P[v] = root of v's component, P[root] = root);
// hooking changes only roots' entries (CAS of the larger root to the
// smaller); path halving writes only ancestors into non-roots.
__device__ __forceinline__ int32_t p_load(const uint16_t* P, int32_t x) {
  return __hip_atomic_load(P + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ int32_t p_root(uint16_t* P, int32_t x) {
  int32_t p = p_load(P, x);
  while (p != x) {
    const int32_t gp = p_load(P, p);
    if (gp == p) return p;
    __hip_atomic_store(P + x, (uint16_t)gp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    x = gp;
    p = p_load(P, x);
  }
  return x;
}
// P[hi]: hi -> lo by a compare-and-swap of the 32-bit word holding it (LDS has
// no 16-bit CAS).  Returns hi on success, else the value P[hi] holds (a
// smaller ancestor).  A failure caused by the other half of the word, which
// only ever decreases, is retried.
__device__ __forceinline__ int32_t p_cas(uint16_t* P, int32_t hi, int32_t lo) {
  uint32_t* word = reinterpret_cast<uint32_t*>(P) + (hi >> 1);
  const int sh = (hi & 1) * 16;
  uint32_t cur = __hip_atomic_load(word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  while (true) {
    const int32_t h = (int32_t)((cur >> sh) & 0xFFFFu);
    if (h != hi) return h;
    const uint32_t nw = (cur & ~(0xFFFFu << sh)) | ((uint32_t)lo << sh);
    if (__hip_atomic_compare_exchange_strong(word, &cur, nw, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_WORKGROUP))
      return hi;
  }
}

// Exclusive prefix sum over the 1024 threads of the workgroup; *total
// receives the sum.  Every thread must call it.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* wsum /* [16] */,
                                                         uint32_t* total) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint32_t x = v;
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  __syncthreads();  // wsum's previous contents are no longer read
  if (lane == 63) wsum[wv] = x;
  __syncthreads();
  uint32_t before = 0, all = 0;
  for (int i = 0; i < 16; ++i) {
    const uint32_t t = wsum[i];
    if (i < wv) before += t;
    all += t;
  }
  *total = all;
  return before + x - v;
}

// One workgroup per graph of `glist` (kSmallN < n <= kMidN, m <= kMidMaxEdges),
// the rounds of Section 2.1 as in k_small_solve, with 10 bytes of LDS per
// vertex: the minimum key per root (u64) and the union-find P (u16), which is
// both the round-start root of every vertex and the parent forest of the
// hooking.  The edges are streamed from memory every round (12 bytes each).
// Thread t owns vertices t + q * kMidBlock (q < kMidPerThread).  Each round:
//   minima   LDS 64-bit atomic min of (w << 32) | local index at the roots of
//            every edge's ends;
//   partner  for every owned root c with a minimum, d = the root at the edge's
//            other end (the edge's loads of all owned roots in flight at
//            once), kept in a register; none when c and d chose each other
//            and d is the smaller (d acts);
//   hooking  CAS of the larger root under the smaller in P, retried from the
//            fresh ancestor the CAS returns; the edge's flag and weight;
//   compress every owned vertex's final root into a register, then P flat
//            again (so no halving store can replace a final value) and the
//            minima of the new roots reset.
// The loop ends when a round selects no edge or at most one component with an
// outgoing edge is left.  Once at most kMidDense such components are left, one
// more pass over the edges takes the minimum key of every pair of them in LDS
// and the remaining rounds run on that table (dense finish, no more passes).  Writes in_mst for the graph's
// edges (zeroed by the caller), total[g] and status[g].
//
// kContracted: the graph is the contraction of batch graph g by its first
// rounds (pre_contract_body): its vertices are the n' = nlist[i] components left,
// its edges the graph's edges (same local indices, so the same keys) with both
// ends given as 16-bit component numbers packed in pairs[poff[i] + j] (a loop
// for an edge inside a component).  The first rounds' edges are already
// flagged and their weight is in total[g]; their count is pcnt[i] and pbad[i]
// flags out-of-range ids, so the status is that of the whole graph.
// (The body of one workgroup, item `item` of A.glist; mbest is the dynamic LDS.)
template <bool kContracted>
__device__ __forceinline__ void mid_solve_body(unsigned long long* mbest /* [n], then P [n] (whole words) */,
                                               const MidArgs& A, int item) {
  __shared__ uint32_t round_sel, round_live;
  __shared__ uint32_t wsum[16];
  __shared__ uint32_t bad;
  __shared__ unsigned long long red_w[kMidBlock / 64];
  __shared__ uint32_t red_c[kMidBlock / 64];

  const int g = A.glist[item];
  const int64_t e0 = A.eoff[g];
  const int64_t m = A.eoff[g + 1] - e0;
  const int32_t n_graph = (int32_t)(A.voff[g + 1] - A.voff[g]);
  const int32_t n = kContracted ? A.nlist[item] : n_graph;
  const int tid = threadIdx.x;
  if (kContracted && (n < 0 || n > A.max_n)) {  // never: each contraction round at least halves the components
    if (tid == 0) A.status[g] = MSTX_ERR_DEVICE;
    return;
  }
  uint16_t* P = reinterpret_cast<uint16_t*>(mbest + n);
  const int32_t* gs = kContracted ? nullptr : A.src + e0;
  const int32_t* gd = kContracted ? nullptr : A.dst + e0;
  const uint32_t* gp = kContracted ? A.pairs + A.poff[item] : nullptr;
  const uint32_t* gw = A.w + e0;
  uint8_t* in_mst = A.in_mst;

  for (int32_t v = tid; v < n; v += kMidBlock) {
    mbest[v] = kKeyNone;
    P[v] = (uint16_t)v;
  }
  if (tid == 0) bad = 0;
  bool my_bad = false;
  unsigned long long my_w = 0;
  uint32_t my_cnt = 0;
  // bit q: owned vertex tid + q * kMidBlock is a root that may still have an
  // outgoing edge (every vertex at the start); their number, uniform
  uint32_t livem = 0;
  for (int q = 0; q < kMidPerThread; ++q)
    if (tid + q * kMidBlock < n) livem |= 1u << q;
  int32_t live_count = n;
  __syncthreads();

  // ends of local edge j from the loaded words (a pair, or src and dst)
  auto split = [&](int32_t& a, int32_t& b) {
    if (kContracted) {
      b = (int32_t)((uint32_t)a >> 16);
      a &= 0xFFFF;
    }
  };

  // (a contracted graph with no component left has only loops)
  for (int round = 0; round < kMaxRounds && m > 0 && n > 0; ++round) {
    if (live_count <= kMidDense) {
      // ---- dense finish.  Numbers 0 .. D-1 for the live roots (block scan),
      // every vertex's number (0xFF: final component), then P and the minima
      // are no longer needed and the pair table takes their place.
      uint8_t* rootnum = reinterpret_cast<uint8_t*>(mbest);  // [n] by root
      uint8_t* vnum = rootnum + n;                           // [n] by vertex
      uint32_t D = 0;
      uint32_t next = block_exclusive_scan((uint32_t)__popc(livem), wsum, &D);
      if (D <= (uint32_t)kMidDense) {  // always: D is the count kept above (uniform)
#pragma unroll
        for (int q = 0; q < kMidPerThread; ++q) {
          const int32_t v = tid + q * kMidBlock;
          if (v < n && P[v] == v) rootnum[v] = ((livem >> q) & 1) ? (uint8_t)next++ : (uint8_t)0xFF;
        }
        __syncthreads();
        for (int32_t v = tid; v < n; v += kMidBlock) vnum[v] = rootnum[P[v]];
        __syncthreads();
        if (D <= 1) break;  // uniform
        const int32_t npairs = (int32_t)(D * (D - 1) / 2);
        unsigned long long* T =
            reinterpret_cast<unsigned long long*>(reinterpret_cast<char*>(mbest) + mid_dense_pairs_at(n));
        unsigned long long* dbest = T + npairs;                    // [D]
        int32_t* dpar = reinterpret_cast<int32_t*>(dbest + D);      // [D] union-find
        int32_t* dcomp = dpar + D;                                  // [D] round-start roots
        for (int32_t x = tid; x < npairs; x += kMidBlock) T[x] = kKeyNone;
        if (tid < (int)D) {
          dpar[tid] = tid;
          dcomp[tid] = tid;
        }
        __syncthreads();
        // the minimum key of every pair of numbers (lo < hi at lo * (2D - lo - 1) / 2 + hi - lo - 1)
        for (int64_t j0 = 0; j0 < m; j0 += (int64_t)kMidUnroll * kMidBlock) {
          int32_t a[kMidUnroll], b[kMidUnroll];
          uint32_t c[kMidUnroll];
#pragma unroll
          for (int q = 0; q < kMidUnroll; ++q) {
            const int64_t j = j0 + q * kMidBlock + tid;
            const int64_t jc = j < m ? j : 0;
            if (kContracted) {
              a[q] = (int32_t)gp[jc];
            } else {
              a[q] = gs[jc];
              b[q] = gd[jc];
            }
            c[q] = gw[jc];
          }
          __asm__ __volatile__("" ::: "memory");
#pragma unroll
          for (int q = 0; q < kMidUnroll; ++q) {
            const int64_t j = j0 + q * kMidBlock + tid;
            if (j >= m) continue;
            split(a[q], b[q]);
            if ((uint32_t)a[q] >= (uint32_t)n || (uint32_t)b[q] >= (uint32_t)n) continue;
            const uint32_t na = vnum[a[q]], nb = vnum[b[q]];
            if (na == 0xFF || nb == 0xFF || na == nb) continue;
            const uint32_t lo = na < nb ? na : nb, hi = na < nb ? nb : na;
            const uint32_t x = lo * (2 * D - lo - 1) / 2 + hi - lo - 1;
            const unsigned long long key = ((unsigned long long)c[q] << 32) | (unsigned long long)j;
            if (key < T[x]) atomicMin(T + x, key);
          }
        }
        __syncthreads();
        // Boruvka rounds on the table, one thread per component
        for (int dr = 0; dr < kMaxRounds; ++dr) {
          if (tid < (int)D) dbest[tid] = kKeyNone;
          if (tid == 0) round_sel = 0;
          __syncthreads();
          for (int32_t x = tid; x < (int32_t)(D * D); x += kMidBlock) {
            const uint32_t lo = (uint32_t)x / D, hi = (uint32_t)x % D;
            if (hi <= lo) continue;
            const unsigned long long key = T[lo * (2 * D - lo - 1) / 2 + hi - lo - 1];
            if (key == kKeyNone) continue;
            const int32_t ra = dcomp[lo], rb = dcomp[hi];
            if (ra == rb) continue;
            if (key < dbest[ra]) atomicMin(dbest + ra, key);
            if (key < dbest[rb]) atomicMin(dbest + rb, key);
          }
          __syncthreads();
          uint32_t dsel = 0;
          if (tid < (int)D && dcomp[tid] == tid && dbest[tid] != kKeyNone) {
            const int32_t c = tid;
            const unsigned long long key = dbest[c];
            const uint32_t j = (uint32_t)key;
            int32_t ea, eb;
            if (kContracted) {
              ea = (int32_t)gp[j];
            } else {
              ea = gs[j];
              eb = gd[j];
            }
            split(ea, eb);
            const int32_t ra = dcomp[vnum[ea]], rb = dcomp[vnum[eb]];
            const int32_t o = (ra == c) ? rb : ra;
            if (!(o < c && dbest[o] == key)) {  // mutual choice: o hooks it
              int32_t x = c, y = o;
              while (true) {
                const int32_t rx = small_root(dpar, x);
                const int32_t ry = small_root(dpar, y);
                if (rx == ry) break;
                const int32_t hi = rx > ry ? rx : ry;
                const int32_t lo = rx > ry ? ry : rx;
                const int32_t old = atomicCAS(dpar + hi, hi, lo);
                if (old == hi) {
                  in_mst[e0 + j] = 1;
                  my_w += (uint32_t)(key >> 32);
                  ++my_cnt;
                  dsel = 1;
                  break;
                }
                if (hi == rx) x = old;
                else y = old;
              }
            }
          }
          dsel = small_wave_sum(dsel);
          if ((tid & 63) == 0 && dsel) atomicAdd(&round_sel, dsel);
          __syncthreads();
          if (round_sel == 0) break;  // uniform
          const int32_t r = tid < (int)D ? small_root(dpar, tid) : 0;
          __syncthreads();
          if (tid < (int)D) {
            dpar[tid] = r;
            dcomp[tid] = r;
          }
          __syncthreads();
        }
        break;
      }
      live_count = (int32_t)D;
    }
    if (tid == 0) {
      round_sel = 0;
      round_live = 0;
    }
    // minima: kMidUnroll edges per thread loaded at once (clamped to edge 0,
    // which exists as m > 0), then offered for the edges that exist
    for (int64_t j0 = 0; j0 < m; j0 += (int64_t)kMidUnroll * kMidBlock) {
      int32_t a[kMidUnroll], b[kMidUnroll];
      uint32_t c[kMidUnroll];
#pragma unroll
      for (int q = 0; q < kMidUnroll; ++q) {
        const int64_t j = j0 + q * kMidBlock + tid;
        const int64_t jc = j < m ? j : 0;
        if (kContracted) {
          a[q] = (int32_t)gp[jc];  // both ends, split below
        } else {
          a[q] = gs[jc];
          b[q] = gd[jc];
        }
        c[q] = gw[jc];
      }
      // keeps every load above issued here, none sunk into the branches below
      // (the edge arrays are not __restrict__, so the clobber pins them)
      __asm__ __volatile__("" ::: "memory");
#pragma unroll
      for (int q = 0; q < kMidUnroll; ++q) {
        const int64_t j = j0 + q * kMidBlock + tid;
        if (j >= m) continue;
        if (kContracted) {
          b[q] = (int32_t)((uint32_t)a[q] >> 16);
          a[q] = a[q] & 0xFFFF;
        }
        if ((uint32_t)a[q] >= (uint32_t)n || (uint32_t)b[q] >= (uint32_t)n) {
          my_bad = true;  // dropped in every round
          continue;
        }
        const int32_t ca = P[a[q]], cb = P[b[q]];
        if (ca == cb) continue;
        const unsigned long long key = ((unsigned long long)c[q] << 32) | (unsigned long long)j;
        if (key < mbest[ca]) atomicMin(mbest + ca, key);
        if (key < mbest[cb]) atomicMin(mbest + cb, key);
      }
    }
    if (my_bad) bad = 1;
    __syncthreads();
    // partner of every owned root (loads clamped to edge 0)
    int32_t d[kMidPerThread];
    uint32_t live = 0;  // owned roots with a minimum edge
    uint32_t hasm = 0;  // which
    {
      int32_t eu[kMidPerThread], ev[kMidPerThread];
#pragma unroll
      for (int q = 0; q < kMidPerThread; ++q) {
        const int32_t c = tid + q * kMidBlock;
        const int32_t cc = c < n ? c : 0;
        const unsigned long long key = mbest[cc];
        const bool has = c < n && P[cc] == c && key != kKeyNone;
        const uint32_t j = has ? (uint32_t)key : 0u;
        if (kContracted) {
          eu[q] = (int32_t)gp[j];
        } else {
          eu[q] = gs[j];
          ev[q] = gd[j];
        }
        d[q] = has ? 0 : -1;
        live += has ? 1u : 0u;
        hasm |= has ? (1u << q) : 0u;
      }
      __asm__ __volatile__("" ::: "memory");
#pragma unroll
      for (int q = 0; q < kMidPerThread; ++q) {
        if (d[q] < 0) continue;
        const int32_t c = tid + q * kMidBlock;
        if (kContracted) {
          ev[q] = (int32_t)((uint32_t)eu[q] >> 16);
          eu[q] = eu[q] & 0xFFFF;
        }
        // a selected edge passed the range check, so its ends index P
        const int32_t pu = P[eu[q]], pv = P[ev[q]];
        const int32_t o = (pu == c) ? pv : pu;
        d[q] = (o < c && mbest[o] == mbest[c]) ? -1 : o;  // mutual choice: o hooks it
      }
    }
    __syncthreads();
    // hooking in LDS
    uint32_t sel = 0;
#pragma unroll
    for (int q = 0; q < kMidPerThread; ++q) {
      if (d[q] < 0) continue;
      const int32_t c = tid + q * kMidBlock;
      const unsigned long long key = mbest[c];
      int32_t x = c, y = d[q];
      while (true) {
        const int32_t rx = p_root(P, x);
        const int32_t ry = p_root(P, y);
        if (rx == ry) break;
        const int32_t hi = rx > ry ? rx : ry;
        const int32_t lo = rx > ry ? ry : rx;
        const int32_t old = p_cas(P, hi, lo);
        if (old == hi) {
          in_mst[e0 + (uint32_t)key] = 1;
          my_w += (uint32_t)(key >> 32);
          ++sel;
          break;
        }
        // the CAS returned a fresh, strictly smaller ancestor: resume there
        if (hi == rx) x = old;
        else y = old;
      }
    }
    my_cnt += sel;
    sel = small_wave_sum(sel);
    live = small_wave_sum(live);
    if ((tid & 63) == 0 && sel) atomicAdd(&round_sel, sel);
    if ((tid & 63) == 0 && live) atomicAdd(&round_live, live);
    __syncthreads();
    // done when no edge was added, or when at most one component with an
    // outgoing edge is left (each added edge merges two of them)
    live_count = (int32_t)((int64_t)round_live - (int64_t)round_sel);
    if (round_sel == 0 || live_count <= 1) break;
    // compression: final roots of the owned vertices into registers (halving
    // stores in P only ever write ancestors, which the walks tolerate), then
    // P flat again
#pragma unroll
    for (int q = 0; q < kMidPerThread; ++q) {
      const int32_t v = tid + q * kMidBlock;
      d[q] = v < n ? p_root(P, v) : 0;
    }
    __syncthreads();
    // a new root may have an outgoing edge only if it had one this round (a
    // root without one was joined by nobody)
    livem = 0;
#pragma unroll
    for (int q = 0; q < kMidPerThread; ++q) {
      const int32_t v = tid + q * kMidBlock;
      if (v >= n) continue;
      P[v] = (uint16_t)d[q];
      if (d[q] == v) {
        mbest[v] = kKeyNone;  // a root of the next round
        livem |= hasm & (1u << q);
      }
    }
    __syncthreads();
  }
  // per-graph totals
  for (int off = 32; off > 0; off >>= 1) {
    my_w += __shfl_xor(my_w, off, 64);
    my_cnt += __shfl_xor(my_cnt, off, 64);
  }
  if ((tid & 63) == 0) {
    red_w[tid >> 6] = my_w;
    red_c[tid >> 6] = my_cnt;
  }
  __syncthreads();
  if (tid == 0) {
    unsigned long long tw = 0;
    uint32_t tc = 0;
    for (int i = 0; i < kMidBlock / 64; ++i) {
      tw += red_w[i];
      tc += red_c[i];
    }
    int64_t count = tc;
    if (kContracted) {
      tw += A.total[g];  // the contraction rounds' edges
      count += A.pcnt[item];
      if (A.pbad[item]) bad = 1;
    }
    A.total[g] = tw;
    int32_t st = (n_graph <= 1 || count == (int64_t)n_graph - 1) ? MSTX_OK : MSTX_DISCONNECTED;
    if (bad) st = MSTX_ERR_VERTEX_RANGE;
    A.status[g] = st;
  }
}

// ------------------------------------------------------- mid-size contraction

static constexpr int kPreBlock = 1024;
static constexpr int kPrePer = kPreMaxN / kPreBlock;  // components per thread: tid + q * kPreBlock
static constexpr int32_t kPreWin = kMaxDynLds / 8;    // minima per LDS window
static constexpr uint16_t kNoLabel = 0xFFFF;          // a final component (no outgoing edge)
static constexpr int kPreHookBatch = 4;               // owned components whose lookups overlap
static_assert(kPrePer <= 64 && kPrePer % kPreHookBatch == 0, "one mask bit per owned component");

// One workgroup per graph of `glist` (n <= kPreMaxN, m <= kMidMaxEdges): the
// rounds of Section 2.1 on densely numbered components while more than
// `target` of them are left, so that the mid-size solve (mid_solve_body in its
// contracted form) can finish the graph in LDS.  Components are numbered
// 0 .. N-1 at the start of every round, so the ends of an edge are its
// components; round 0 reads the caller's edges (ids checked against [0, n)),
// later rounds the 16-bit pairs the previous round wrote.  Each round:
//   minima    windows of kPreWin components in LDS (64-bit atomic min of
//             (w << 32) | local index), each flushed to the graph's scratch;
//   hooking   u16 union-find P[N] in LDS, CAS of the larger root under the
//             smaller (partners are plain edge ends: no lookup races the
//             hooks; an edge two components chose is added by whichever CAS
//             wins), the edge's flag, weight and count;
//   numbering P flat (final roots through the scratch), then consecutive
//             numbers for the roots that had a minimum edge (block scan); a
//             root without one is a final component;
//   edges     pairs[poff[i] + j] <- the new numbers of both ends, or a loop
//             (0, 0) for an edge inside a final component or out of range.
// Outputs: nlist[i] = components left (their numbers in the pairs), pcnt[i] =
// edges added, pbad[i] = out-of-range ids seen, total[g] = their weight.
// (The body of one workgroup, item `item` of A.glist; wbest is the dynamic LDS.)
__device__ __forceinline__ void pre_contract_body(unsigned long long* wbest /* [kPreWin] minima window */,
                                                  const PreArgs& A, int item) {
  uint16_t* P = reinterpret_cast<uint16_t*>(wbest);  // [N] union-find, then the new numbers
  __shared__ uint32_t wsum[kPreBlock / 64];
  __shared__ uint32_t round_sel;
  __shared__ uint32_t bad;
  __shared__ unsigned long long red_w[kPreBlock / 64];
  __shared__ uint32_t red_c[kPreBlock / 64];

  const int i = item;
  const int g = A.glist[i];
  const int64_t e0 = A.eoff[g];
  const int64_t m = A.eoff[g + 1] - e0;
  const int32_t n = (int32_t)(A.voff[g + 1] - A.voff[g]);
  const int tid = threadIdx.x;
  if (n > kPreMaxN) {  // never: the host sends no such graph
    if (tid == 0) A.nlist[i] = -1;
    return;
  }
  unsigned long long* gbest = A.scratch + A.soff[i];  // [n]
  int32_t* gtmp = reinterpret_cast<int32_t*>(gbest);  // [n], once the minima are read
  const int32_t* gs = A.src + e0;
  const int32_t* gd = A.dst + e0;
  const uint32_t* gw = A.w + e0;
  uint32_t* gp = A.pairs + A.poff[i];
  if (tid == 0) bad = 0;
  bool my_bad = false;
  unsigned long long my_w = 0;
  uint32_t my_cnt = 0;
  int32_t N = n;
  bool from_input = true;
  __syncthreads();

  // ends of edge j (clamped loads issued by the caller): from the caller's
  // arrays, range-checked, or unpacked from a pair; false for a dropped edge
  auto ends = [&](int32_t& a, int32_t& b) -> bool {
    if (from_input) {
      if ((uint32_t)a >= (uint32_t)n || (uint32_t)b >= (uint32_t)n) {
        my_bad = true;
        return false;
      }
      return true;
    }
    b = (int32_t)((uint32_t)a >> 16);
    a &= 0xFFFF;
    return true;
  };

  for (int round = 0; round < kMaxRounds && N > A.target && m > 0; ++round) {
    // minima, one window of components at a time.  The first pass of round 0
    // reads the caller's arrays and writes every edge's ends as a pair (the
    // vertices are round 0's components; a loop for an out-of-range edge), so
    // every later step reads 4-byte pairs instead of src and dst.
    for (int32_t lo = 0; lo < N; lo += kPreWin) {
      const int32_t span = min(N - lo, kPreWin);
      for (int32_t c = tid; c < span; c += kPreBlock) wbest[c] = kKeyNone;
      __syncthreads();
      for (int64_t j0 = 0; j0 < m; j0 += (int64_t)kMidUnroll * kPreBlock) {
        int32_t a[kMidUnroll], b[kMidUnroll];
        uint32_t c[kMidUnroll];
#pragma unroll
        for (int q = 0; q < kMidUnroll; ++q) {
          const int64_t j = j0 + q * kPreBlock + tid;
          const int64_t jc = j < m ? j : 0;
          if (from_input) {
            a[q] = gs[jc];
            b[q] = gd[jc];
          } else {
            a[q] = (int32_t)gp[jc];
          }
          c[q] = gw[jc];
        }
        __asm__ __volatile__("" ::: "memory");
#pragma unroll
        for (int q = 0; q < kMidUnroll; ++q) {
          const int64_t j = j0 + q * kPreBlock + tid;
          if (j >= m) continue;
          const bool ok = ends(a[q], b[q]);
          if (from_input) gp[j] = ok ? ((uint32_t)a[q] | ((uint32_t)b[q] << 16)) : 0u;
          if (!ok || a[q] == b[q]) continue;
          const unsigned long long key = ((unsigned long long)c[q] << 32) | (unsigned long long)j;
          const uint32_t ra = (uint32_t)(a[q] - lo), rb = (uint32_t)(b[q] - lo);
          if (ra < (uint32_t)span && key < wbest[ra]) atomicMin(wbest + ra, key);
          if (rb < (uint32_t)span && key < wbest[rb]) atomicMin(wbest + rb, key);
        }
      }
      __syncthreads();
      for (int32_t c = tid; c < span; c += kPreBlock) gbest[lo + c] = wbest[c];
      __syncthreads();
      from_input = false;  // the pairs are written (uniform)
    }
    if (my_bad) bad = 1;
    // hooking over the N components
    for (int32_t c = tid; c < N; c += kPreBlock) P[c] = (uint16_t)c;
    if (tid == 0) round_sel = 0;
    __syncthreads();
    uint64_t had = 0;  // bit q: component tid + q * kPreBlock had a minimum edge
    uint32_t sel = 0;
    for (int q0 = 0; q0 < kPrePer && tid + q0 * kPreBlock < N; q0 += kPreHookBatch) {
      unsigned long long key[kPreHookBatch];
      int32_t eu[kPreHookBatch], ev[kPreHookBatch], d[kPreHookBatch];
      bool has[kPreHookBatch];
#pragma unroll
      for (int r = 0; r < kPreHookBatch; ++r) {
        const int32_t c = tid + (q0 + r) * kPreBlock;
        key[r] = gbest[c < N ? c : 0];
      }
#pragma unroll
      for (int r = 0; r < kPreHookBatch; ++r) {
        const int32_t c = tid + (q0 + r) * kPreBlock;
        has[r] = c < N && key[r] != kKeyNone;
        const uint32_t j = has[r] ? (uint32_t)key[r] : 0u;  // a selected edge exists, so m > 0
        if (from_input) {
          eu[r] = gs[j];
          ev[r] = gd[j];
        } else {
          eu[r] = (int32_t)gp[j];
        }
      }
      __asm__ __volatile__("" ::: "memory");
#pragma unroll
      for (int r = 0; r < kPreHookBatch; ++r) {
        const int32_t c = tid + (q0 + r) * kPreBlock;
        if (!from_input) {
          ev[r] = (int32_t)((uint32_t)eu[r] >> 16);
          eu[r] &= 0xFFFF;
        }
        d[r] = (eu[r] == c) ? ev[r] : eu[r];  // a selected edge passed the range check
      }
#pragma unroll
      for (int r = 0; r < kPreHookBatch; ++r) {
        if (!has[r]) continue;
        had |= 1ull << (q0 + r);
        // no mutual-choice check (it would cost a third dependent load): when
        // c and d chose each other both threads try the same CAS, one wins,
        // and the other then finds both ends under one root
        const int32_t c = tid + (q0 + r) * kPreBlock;
        int32_t x = c, y = d[r];
        while (true) {
          const int32_t rx = p_root(P, x);
          const int32_t ry = p_root(P, y);
          if (rx == ry) break;
          const int32_t hi = rx > ry ? rx : ry;
          const int32_t lo = rx > ry ? ry : rx;
          const int32_t old = p_cas(P, hi, lo);
          if (old == hi) {
            A.in_mst[e0 + (uint32_t)key[r]] = 1;
            my_w += (uint32_t)(key[r] >> 32);
            ++sel;
            break;
          }
          if (hi == rx) x = old;
          else y = old;
        }
      }
    }
    my_cnt += sel;
    sel = small_wave_sum(sel);
    if ((tid & 63) == 0 && sel) atomicAdd(&round_sel, sel);
    __syncthreads();
    // flatten: final roots through the scratch (the minima are read), so no
    // halving store can replace a final value
    for (int32_t c = tid; c < N; c += kPreBlock) gtmp[c] = p_root(P, c);
    __syncthreads();
    for (int32_t c = tid; c < N; c += kPreBlock) P[c] = (uint16_t)gtmp[c];
    __syncthreads();
    // consecutive numbers for the roots that had a minimum edge
    uint32_t roots = 0;
#pragma unroll 8
    for (int q = 0; q < kPrePer; ++q) {
      const int32_t c = tid + q * kPreBlock;
      if (c < N && P[c] == c && ((had >> q) & 1)) ++roots;
    }
    uint32_t n_next = 0;
    uint32_t next = block_exclusive_scan(roots, wsum, &n_next);
#pragma unroll 8
    for (int q = 0; q < kPrePer; ++q) {
      const int32_t c = tid + q * kPreBlock;
      if (c < N && P[c] == c) gtmp[c] = ((had >> q) & 1) ? (int32_t)next++ : -1;
    }
    __syncthreads();
    for (int32_t c = tid; c < N; c += kPreBlock) {
      const int32_t l = gtmp[P[c]];
      P[c] = l < 0 ? kNoLabel : (uint16_t)l;
    }
    __syncthreads();
    // the edges as pairs of the new numbers
    for (int64_t j0 = 0; j0 < m; j0 += (int64_t)kMidUnroll * kPreBlock) {
      int32_t a[kMidUnroll], b[kMidUnroll];
#pragma unroll
      for (int q = 0; q < kMidUnroll; ++q) {
        const int64_t j = j0 + q * kPreBlock + tid;
        const int64_t jc = j < m ? j : 0;
        if (from_input) {
          a[q] = gs[jc];
          b[q] = gd[jc];
        } else {
          a[q] = (int32_t)gp[jc];
        }
      }
      __asm__ __volatile__("" ::: "memory");
#pragma unroll
      for (int q = 0; q < kMidUnroll; ++q) {
        const int64_t j = j0 + q * kPreBlock + tid;
        if (j >= m) continue;
        uint32_t pr = 0;
        if (ends(a[q], b[q])) {
          const uint32_t la = P[a[q]], lb = P[b[q]];
          if (la != kNoLabel && lb != kNoLabel) pr = la | (lb << 16);
        }
        gp[j] = pr;
      }
    }
    __syncthreads();
    N = (int32_t)n_next;
    from_input = false;
  }
  if (from_input && m > 0) {
    // no round ran (at most `target` vertices): the ends as they are
    for (int64_t j = tid; j < m; j += kPreBlock) {
      int32_t a = gs[j], b = gd[j];
      gp[j] = ends(a, b) ? ((uint32_t)a | ((uint32_t)b << 16)) : 0u;
    }
    if (my_bad) bad = 1;
  }
  // no edges at all: every vertex is a final component, none is left to solve
  if (m == 0) N = 0;
  for (int off = 32; off > 0; off >>= 1) {
    my_w += __shfl_xor(my_w, off, 64);
    my_cnt += __shfl_xor(my_cnt, off, 64);
  }
  if ((tid & 63) == 0) {
    red_w[tid >> 6] = my_w;
    red_c[tid >> 6] = my_cnt;
  }
  __syncthreads();
  if (tid == 0) {
    unsigned long long tw = 0;
    uint32_t tc = 0;
    for (int k = 0; k < kPreBlock / 64; ++k) {
      tw += red_w[k];
      tc += red_c[k];
    }
    A.total[g] = tw;
    A.pcnt[i] = (int32_t)tc;
    A.pbad[i] = bad;
    A.nlist[i] = N;
  }
}

// ------------------------------------------------------- one launch per batch

// Every graph of a batch that one workgroup solves, in one launch: items
// [0, ncon) are contracted (pre_contract_body's rounds, then the contracted
// mid-size solve, in the same workgroup), [ncon, ncon + nmid) mid-size and
// the rest small.  Each class comes most edges first, so the longest
// workgroups start first and the small graphs fill the tail.
__global__ void __launch_bounds__(kMidBlock) k_batch_solve(BatchSolveArgs B) {
  extern __shared__ unsigned long long dyn_lds[];
  const int i = blockIdx.x;
  if (i < B.ncon) {
    pre_contract_body(dyn_lds, B.pre, i);
    __syncthreads();  // the contraction's outputs and LDS, then the mid-size solve's
    mid_solve_body<true>(dyn_lds, B.con, i);
  } else if (i < B.ncon + B.nmid) {
    mid_solve_body<false>(dyn_lds, B.mid, i - B.ncon);
  } else {
    const MidArgs& S = B.small;
    small_solve_body(dyn_lds, i - B.ncon - B.nmid, S.glist, S.voff, S.eoff, 0, 0, S.src, S.dst, S.w, S.in_mst,
                     S.total, S.status, nullptr, (uint32_t)kMaxDynLds);
  }
}

// Union of the chunk's graphs glist[0..ng): chunk edge p belongs to graph k with
// cedge[k] <= p < cedge[k+1]; its ends become union ids cvert[k] + local id.
// An end outside [0, n_g) makes the edge a self-loop at cvert[k] and flags the
// graph.  w is copied so the union's edges are contiguous.
__global__ void __launch_bounds__(256) k_gather(const int32_t* __restrict__ glist, int ng,
                                                const int64_t* __restrict__ voff,
                                                const int64_t* __restrict__ eoff,
                                                const int64_t* __restrict__ cvert,
                                                const int64_t* __restrict__ cedge,
                                                const int32_t* __restrict__ src,
                                                const int32_t* __restrict__ dst,
                                                const uint32_t* __restrict__ w, int32_t* __restrict__ gsrc,
                                                int32_t* __restrict__ gdst, uint32_t* __restrict__ gw,
                                                int32_t* __restrict__ gbad) {
  const int64_t total = cedge[ng];
  const int64_t per_block = 4096;
  for (int64_t b0 = (int64_t)blockIdx.x * per_block; b0 < total; b0 += (int64_t)gridDim.x * per_block) {
    // graph of this block's first edge (binary search), then forward steps per edge
    __shared__ int k0s;
    if (threadIdx.x == 0) {
      int lo = 0, hi = ng - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (cedge[mid] <= b0) lo = mid;
        else hi = mid - 1;
      }
      k0s = lo;
    }
    __syncthreads();
    const int k0 = k0s;
    __syncthreads();
    const int64_t b1 = min(total, b0 + per_block);
    for (int64_t p = b0 + threadIdx.x; p < b1; p += blockDim.x) {
      int k = k0;
      while (cedge[k + 1] <= p) ++k;
      const int g = glist[k];
      const int64_t j = eoff[g] + (p - cedge[k]);
      const int32_t n = (int32_t)(voff[g + 1] - voff[g]);
      int32_t a = src[j], b = dst[j];
      if ((uint32_t)a >= (uint32_t)n || (uint32_t)b >= (uint32_t)n) {
        gbad[k] = 1;
        a = b = 0;
      }
      gsrc[p] = (int32_t)(cvert[k] + a);
      gdst[p] = (int32_t)(cvert[k] + b);
      gw[p] = w[j];
    }
  }
}

// Chunk graph k, slice y of `slice` edges (a 2-D grid: large graphs get many
// workgroups): copies the union's flags back to the caller's in_mst
// range of graph glist[k] and adds the weight and count of the marked edges
// of the slice to acc_w[k], acc_c[k] (zeroed by the caller; one atomic per
// workgroup).
static constexpr int64_t kEpilogueSlice = 16384;  // edges per workgroup (at least)
static constexpr int kEpilogueUnroll = 8;          // edges per thread in flight
__global__ void __launch_bounds__(256) k_graph_epilogue(const int32_t* __restrict__ glist, int64_t slice,
                                                        const int64_t* __restrict__ eoff,
                                                        const int64_t* __restrict__ cedge,
                                                        const uint8_t* cin_mst, const uint32_t* gw,
                                                        uint8_t* __restrict__ in_mst,
                                                        unsigned long long* __restrict__ acc_w,
                                                        uint32_t* __restrict__ acc_c) {
  __shared__ unsigned long long rw[4];
  __shared__ uint32_t rc[4];
  const int k = blockIdx.x;
  const int64_t p_first = cedge[k] + (int64_t)blockIdx.y * slice;
  const int64_t p_end = min(cedge[k + 1], p_first + slice);
  if (p_first >= p_end) return;  // uniform: the graph has fewer slices
  const int64_t to = eoff[glist[k]] - cedge[k];  // caller index = chunk index + to
  unsigned long long sw = 0;
  uint32_t cnt = 0;
  // kEpilogueUnroll edges per thread with their loads (clamped to the
  // slice's first edge) in flight together; the memory clobbers keep them
  // issued before the first use
  for (int64_t p0 = p_first + threadIdx.x; p0 < p_end; p0 += kEpilogueUnroll * 256) {
    uint8_t f[kEpilogueUnroll];
    uint32_t wq[kEpilogueUnroll];
#pragma unroll
    for (int q = 0; q < kEpilogueUnroll; ++q) {
      const int64_t p = p0 + q * 256;
      const int64_t pc = p < p_end ? p : p_first;
      f[q] = cin_mst[pc];
      wq[q] = gw[pc];
    }
    __asm__ __volatile__("" ::: "memory");
#pragma unroll
    for (int q = 0; q < kEpilogueUnroll; ++q) {
      const int64_t p = p0 + q * 256;
      if (p >= p_end) continue;
      in_mst[p + to] = f[q];
      if (f[q]) {
        sw += wq[q];
        ++cnt;
      }
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    sw += __shfl_xor(sw, off, 64);
    cnt += __shfl_xor(cnt, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    rw[threadIdx.x >> 6] = sw;
    rc[threadIdx.x >> 6] = cnt;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned long long tw = rw[0] + rw[1] + rw[2] + rw[3];
    const uint32_t tc = rc[0] + rc[1] + rc[2] + rc[3];
    if (tw) atomicAdd(acc_w + k, tw);
    if (tc) atomicAdd(acc_c + k, tc);
  }
}

// Per chunk graph: total[g] and status[g] from the accumulated sums.
__global__ void __launch_bounds__(256) k_graph_status(const int32_t* __restrict__ glist, int ng,
                                                      const int64_t* __restrict__ voff,
                                                      const unsigned long long* __restrict__ acc_w,
                                                      const uint32_t* __restrict__ acc_c,
                                                      const int32_t* __restrict__ gbad,
                                                      unsigned long long* __restrict__ total_out,
                                                      int32_t* __restrict__ status_out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= ng) return;
  const int g = glist[k];
  const int64_t n = voff[g + 1] - voff[g];
  total_out[g] = acc_w[k];
  int32_t st = (n <= 1 || (int64_t)acc_c[k] == n - 1) ? MSTX_OK : MSTX_DISCONNECTED;
  if (gbad[k]) st = MSTX_ERR_VERTEX_RANGE;
  status_out[g] = st;
}

hipError_t configure_batched_kernels() {
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_small_solve),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxDynLds);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_batch_solve), hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)kMaxDynLds);
}

hipError_t launch_batch_solve(const BatchSolveArgs& B, int nsmall, hipStream_t s) {
  const int num = B.ncon + B.nmid + nsmall;
  if (num <= 0) return hipSuccess;
  if (B.ncon > 0 && (B.pre.target < 1 || B.pre.target > kMidN || B.con.max_n != B.pre.target))
    return hipErrorInvalidValue;
  if (B.nmid > 0 && (B.mid.max_n < 1 || B.mid.max_n > kMidN)) return hipErrorInvalidValue;
  static_assert(kSmallSolveLds <= kMaxDynLds && kSmallBlock == kMidBlock && kPreBlock == kMidBlock,
                "one workgroup shape and LDS allocation serve every class");
  k_batch_solve<<<num, kMidBlock, kMaxDynLds, s>>>(B);
  return hipGetLastError();
}



hipError_t launch_small_solve_single(int32_t n, int64_t m, const int32_t* src, const int32_t* dst,
                                     const uint32_t* w, uint8_t* in_mst, unsigned long long* total,
                                     int32_t* status, int64_t* stats, hipStream_t s) {
  // the vertex state, and the edges too when both fit the workgroup's LDS
  const size_t state = ((size_t)16 * (size_t)n + 15) & ~(size_t)15;
  const size_t lds = state + 12 * (size_t)m <= (size_t)kMaxDynLds ? state + 12 * (size_t)m : (size_t)16 * n;
  k_small_solve<<<1, kSmallBlock, lds, s>>>(nullptr, nullptr, nullptr, n, m, src, dst, w, in_mst, total, status,
                                             stats, (uint32_t)lds);
  return hipGetLastError();
}

hipError_t launch_gather(const int32_t* glist, int ng, const int64_t* voff, const int64_t* eoff,
                         const int64_t* cvert, const int64_t* cedge, int64_t chunk_edges, const int32_t* src,
                         const int32_t* dst, const uint32_t* w, int32_t* gsrc, int32_t* gdst, uint32_t* gw,
                         int32_t* gbad, hipStream_t s) {
  if (ng <= 0 || chunk_edges <= 0) return hipSuccess;
  const int64_t blocks = (chunk_edges + 4095) / 4096;
  const int grid = (int)(blocks < 8192 ? blocks : 8192);
  k_gather<<<grid, 256, 0, s>>>(glist, ng, voff, eoff, cvert, cedge, src, dst, w, gsrc, gdst, gw, gbad);
  return hipGetLastError();
}

hipError_t launch_graph_epilogue(const int32_t* glist, int ng, const int64_t* voff, const int64_t* eoff,
                                 const int64_t* cedge, int64_t max_graph_m, const uint8_t* cin_mst,
                                 const uint32_t* gw, const int32_t* gbad, uint8_t* in_mst,
                                 unsigned long long* acc_w, uint32_t* acc_c, unsigned long long* total,
                                 int32_t* status, hipStream_t s) {
  if (ng <= 0) return hipSuccess;
  hipError_t e = hipMemsetAsync(acc_w, 0, 8 * (size_t)ng, s);
  if (e == hipSuccess) e = hipMemsetAsync(acc_c, 0, 4 * (size_t)ng, s);
  if (e != hipSuccess) return e;
  // at most 65535 slices per graph (the grid's y limit)
  const int64_t slice = std::max<int64_t>(kEpilogueSlice, (max_graph_m + 65534) / 65535);
  const int64_t slices = std::max<int64_t>(1, (max_graph_m + slice - 1) / slice);
  k_graph_epilogue<<<dim3(ng, (unsigned)slices), 256, 0, s>>>(glist, slice, eoff, cedge, cin_mst, gw, in_mst,
                                                               acc_w, acc_c);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_graph_status<<<(ng + 255) / 256, 256, 0, s>>>(glist, ng, voff, acc_w, acc_c, gbad, total, status);
  return hipGetLastError();
}

}  // namespace mstx
