// mstx_batched.hip -- kernels of the batched solve (many independent graphs in one call).
//
// The minimum spanning forest of a disjoint union of graphs is the union of
// their forests, and Boruvka never merges components of different graphs, so
// a batch is solved in two parts:
//
//   * graphs with at most kSmallN vertices: one workgroup per graph runs every
//     Boruvka round of Section 2.1 with the vertex state in LDS (component of
//     each vertex, union-find parents, minimum keys); rounds are separated by
//     workgroup barriers only, so thousands of small graphs proceed
//     independently and in parallel;
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
  extern __shared__ unsigned long long sbest[];  // [n], then comp [n], par [n], the edge cache
  __shared__ uint32_t round_sel;
  __shared__ uint32_t bad;
  __shared__ unsigned long long red_w[kSmallBlock / 64];
  __shared__ uint32_t red_c[kSmallBlock / 64];
  __shared__ uint32_t round_live, round_nonisolated;

  const int g = glist ? glist[blockIdx.x] : 0;
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
    if (stats) {
      nonisolated = small_wave_sum(nonisolated);
      if ((tid & 63) == 0 && nonisolated) atomicAdd(&round_nonisolated, nonisolated);
    }
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
    if (round_sel == 0) break;
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
__global__ void __launch_bounds__(256) k_graph_epilogue(const int32_t* __restrict__ glist, int64_t slice,
                                                        const int64_t* __restrict__ eoff,
                                                        const int64_t* __restrict__ cedge,
                                                        const uint8_t* __restrict__ cin_mst,
                                                        const uint32_t* __restrict__ gw,
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
  for (int64_t p = p_first + threadIdx.x; p < p_end; p += blockDim.x) {
    const uint8_t f = cin_mst[p];
    in_mst[p + to] = f;
    if (f) {
      sw += gw[p];
      ++cnt;
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
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_small_solve),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxDynLds);
}

hipError_t launch_small_solve(const int32_t* glist, int num, const int64_t* voff, const int64_t* eoff,
                              const int32_t* src, const int32_t* dst, const uint32_t* w, uint8_t* in_mst,
                              unsigned long long* total, int32_t* status, hipStream_t s) {
  if (num <= 0) return hipSuccess;
  k_small_solve<<<num, kSmallBlock, kSmallSolveLds, s>>>(glist, voff, eoff, 0, 0, src, dst, w, in_mst, total,
                                                          status, nullptr, (uint32_t)kSmallSolveLds);
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
