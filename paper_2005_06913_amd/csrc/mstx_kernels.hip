// mstx_kernels.hip -- device kernels of the parallel Boruvka MST for CDNA4 (gfx950).
//
// One Boruvka round (Durbhakula, arXiv 2005.06913, Section 2.1; CAS union of
// Section 2.2.2) is five kernels, each a global barrier for the next:
//
//   scan      every live edge: labels of both ends at this round; drop it if
//             internal (the paper's "covered" edge); otherwise lower the
//             per-component minimum key of both ends.  The key packs
//             (w << 32) | e, so the order is strict and ties cannot occur.
//             Rounds >= 1 also compact the survivors in place.
//   hook      every component with a minimum: unite its root with the root of
//             the other end's component by compare-and-swap of the larger
//             root's parent to the smaller root; the winner marks the edge.
//   compress  pointer jumping: every component finds its root; a wave ballot
//             records which components are roots of non-isolated trees.
//   finalize  one workgroup: exclusive scan of the root counts (dense new
//             labels), per-round totals (live edges, edges added, weight).
//   relabel   old label -> new label map; reset parent[] and the minima.
//
// Layout: vertex state is structure-of-arrays in HBM (best[] u64, parent[],
// root_of[] i32, one label map per round in a pool).  The edge stream of
// round 0 is the caller's src/dst/w arrays; from round 1 on it is a record
// stream {a, b, w, e} (16 B, one dwordx4 per edge) split into fixed segments,
// one per workgroup, compacted in place each round.
//
// Atomics: device-scope 64-bit atomics on gfx950 execute at the memory side,
// so every global atomicMin is preceded by a plain load that skips it when
// the stored key is already smaller (values only decrease, so a stale load is
// only ever too large and never skips a needed update).  When the current
// component count fits in LDS, minima are kept per workgroup in LDS and
// flushed once.  No kernel uses same-address global atomics: per-block
// partial sums go to arrays that the single-workgroup finalize reduces.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mstx_internal.h"

namespace mstx {

static constexpr int kBlock = 256;    // threads per workgroup for the streaming kernels
static constexpr int kPerThread = 4;  // records per thread per tile in the segmented scan
static constexpr int kTile = kBlock * kPerThread;
static constexpr int kWaves = kBlock / 64;

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ uint64_t make_key(uint32_t w, uint32_t e) {
  return ((uint64_t)w << 32) | (uint64_t)e;
}

// Lower best[c] to key; the plain load filters the memory-side atomic.
__device__ __forceinline__ void lower_global(unsigned long long* best, int32_t c, uint64_t key) {
  if (key < best[c]) atomicMin(best + c, (unsigned long long)key);
}

__device__ __forceinline__ void lower_lds(unsigned long long* lbest, int32_t c, uint64_t key) {
  if (key < lbest[c]) atomicMin(lbest + c, (unsigned long long)key);
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

__device__ __forceinline__ uint64_t lanemask_lt() {
  const int l = lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum over a 256-thread block; result valid in every thread.
template <typename T>
__device__ __forceinline__ T block_sum(T v, T* scratch /* [kWaves] */) {
  v = wave_sum(v);
  __syncthreads();
  if (lane_id() == 0) scratch[threadIdx.x >> 6] = v;
  __syncthreads();
  T s = 0;
#pragma unroll
  for (int i = 0; i < kWaves; ++i) s += scratch[i];
  return s;
}

__device__ __forceinline__ int32_t ld_agent(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(int32_t* p, int32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// --------------------------------------------------------------------- init

// best[0..n) <- none, parent[c] <- c, state counters for round 0.
__global__ void __launch_bounds__(kBlock) k_init(int32_t n, uint32_t m, unsigned long long* best,
                                                 int32_t* parent, DevState* st) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += stride) {
    best[c] = kKeyNone;
    parent[c] = (int32_t)c;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->n[0] = n;
    st->lab_off[0] = 0;
    st->err = 0;
    st->err_internal = 0;
    st->edges_added = 0;
    (void)m;
  }
}

__global__ void __launch_bounds__(kBlock) k_fill_u64(unsigned long long* p, int64_t count, unsigned long long v) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) p[i] = v;
}

// ---------------------------------------------------------- round 0: scan

// Edge loop of round 0 over the caller's arrays.  Labels are the vertex ids.
// Out-of-range ids set st->err and the edge is skipped.  part_live[block] =
// number of non-loop in-range edges this block saw.
template <bool kLds>
__global__ void __launch_bounds__(kBlock) k_scan_first(const int32_t* __restrict__ src,
                                                       const int32_t* __restrict__ dst,
                                                       const uint32_t* __restrict__ w, uint32_t m,
                                                       int32_t n, unsigned long long* __restrict__ best,
                                                       uint32_t* __restrict__ part_live,
                                                       DevState* __restrict__ st) {
  extern __shared__ unsigned long long lbest[];  // n entries when kLds
  __shared__ uint32_t red[kWaves];
  if (kLds) {
    for (int32_t c = threadIdx.x; c < n; c += kBlock) lbest[c] = kKeyNone;
    __syncthreads();
  }
  uint32_t live = 0;
  bool bad = false;
  const uint32_t stride = gridDim.x * kBlock;
  for (uint32_t e = blockIdx.x * kBlock + threadIdx.x; e < m; e += stride) {
    const int32_t a = src[e];
    const int32_t b = dst[e];
    const uint32_t we = w[e];
    if ((uint32_t)a >= (uint32_t)n || (uint32_t)b >= (uint32_t)n) {
      bad = true;
      continue;
    }
    if (a == b) continue;
    ++live;
    const uint64_t key = make_key(we, e);
    if (kLds) {
      lower_lds(lbest, a, key);
      lower_lds(lbest, b, key);
    } else {
      lower_global(best, a, key);
      lower_global(best, b, key);
    }
  }
  if (bad) st->err = 1;
  if (kLds) {
    __syncthreads();
    for (int32_t c = threadIdx.x; c < n; c += kBlock) {
      const unsigned long long v = lbest[c];
      if (v != kKeyNone) lower_global(best, c, v);
    }
  }
  live = block_sum(live, red);
  if (threadIdx.x == 0) part_live[blockIdx.x] = live;
}

// ------------------------------------------------- rounds >= 1: scan+compact

// Segment s holds records [s*seg_cap, s*seg_cap + seg_cnt[s]) of the record
// stream.  In round 1 (kFromInput) segment s is instead the caller's edges
// [s*seg_cap, min((s+1)*seg_cap, m)) with labels lab[src], lab[dst].  Every
// surviving edge (ends in different components) lowers the minima of both
// components and is written back compacted to the front of its segment.
// Reads of a tile complete before the barrier that precedes its writes, and
// writes never pass the tile being read, so compaction in place is safe.
template <bool kFromInput, bool kLds>
__global__ void __launch_bounds__(kBlock) k_scan_seg(
    int round, const int32_t* __restrict__ src, const int32_t* __restrict__ dst,
    const uint32_t* __restrict__ w, uint32_t m, const int32_t* __restrict__ labpool, uint4* rec,
    uint32_t* __restrict__ seg_cnt, uint32_t seg_cap, int32_t nseg,
    unsigned long long* __restrict__ best, const DevState* __restrict__ st) {
  extern __shared__ unsigned long long lbest[];  // nr entries when kLds
  __shared__ uint32_t wave_tot[2][kWaves];
  const int32_t nr = st->n[round];
  const int32_t* __restrict__ lab = labpool + st->lab_off[round - 1];  // labels of round r-1 -> r
  if (kLds) {
    for (int32_t c = threadIdx.x; c < nr; c += kBlock) lbest[c] = kKeyNone;
    __syncthreads();
  }
  const int wave = threadIdx.x >> 6;
  const uint64_t lt = lanemask_lt();
  int parity = 0;
  for (int32_t s = blockIdx.x; s < nseg; s += gridDim.x) {
    const uint64_t base = (uint64_t)s * seg_cap;
    uint32_t count;
    if (kFromInput) {
      count = base >= m ? 0u : (uint32_t)min((uint64_t)seg_cap, (uint64_t)m - base);
    } else {
      count = seg_cnt[s];
    }
    uint32_t wpos = 0;
    for (uint32_t t = 0; t < count; t += kTile) {
      uint4 r[kPerThread];
      bool live[kPerThread];
#pragma unroll
      for (int k = 0; k < kPerThread; ++k) {
        const uint32_t j = t + k * kBlock + threadIdx.x;
        live[k] = false;
        if (j < count) {
          int32_t a, b;
          uint32_t we, e;
          if (kFromInput) {
            e = (uint32_t)(base + j);
            a = lab[src[e]];
            b = lab[dst[e]];
            we = w[e];
          } else {
            const uint4 x = rec[base + j];
            a = lab[(int32_t)x.x];
            b = lab[(int32_t)x.y];
            we = x.z;
            e = x.w;
          }
          r[k] = make_uint4((uint32_t)a, (uint32_t)b, we, e);
          // a live record never touches an isolated (label -1) component
          live[k] = (a != b) && ((a | b) >= 0);
          if (live[k]) {
            const uint64_t key = make_key(we, e);
            if (kLds) {
              lower_lds(lbest, a, key);
              lower_lds(lbest, b, key);
            } else {
              lower_global(best, a, key);
              lower_global(best, b, key);
            }
          }
        }
      }
      // wave-level compaction offsets, slot-major within the wave
      uint32_t my_off[kPerThread];
      uint32_t run = 0;
#pragma unroll
      for (int k = 0; k < kPerThread; ++k) {
        const uint64_t mask = __ballot(live[k]);
        my_off[k] = run + (uint32_t)__popcll(mask & lt);
        run += (uint32_t)__popcll(mask);
      }
      if (lane_id() == 0) wave_tot[parity][wave] = run;
      __syncthreads();  // all reads of this tile are done past this point
      uint32_t wave_off = 0, tile_tot = 0;
#pragma unroll
      for (int i = 0; i < kWaves; ++i) {
        const uint32_t v = wave_tot[parity][i];
        wave_off += (i < wave) ? v : 0u;
        tile_tot += v;
      }
#pragma unroll
      for (int k = 0; k < kPerThread; ++k) {
        if (live[k]) rec[base + wpos + wave_off + my_off[k]] = r[k];
      }
      wpos += tile_tot;
      parity ^= 1;
    }
    if (threadIdx.x == 0) seg_cnt[s] = wpos;
  }
  if (kLds) {
    __syncthreads();
    for (int32_t c = threadIdx.x; c < nr; c += kBlock) {
      const unsigned long long v = lbest[c];
      if (v != kKeyNone) lower_global(best, c, v);
    }
  }
}

// -------------------------------------------------------------------- hook

// Root of x with path halving.  Loads and stores are agent-scope atomics so a
// root changed by another workgroup's CAS is seen.  Every halving store
// writes an ancestor, and only to a non-root, so it never undoes a union.
__device__ __forceinline__ int32_t hook_find(int32_t* parent, int32_t x) {
  while (true) {
    const int32_t p = ld_agent(parent + x);
    if (p == x) return x;
    const int32_t gp = ld_agent(parent + p);
    if (gp == p) return p;
    st_agent(parent + x, gp);
    x = gp;
  }
}

// For each component c with a minimum edge e = low32(best[c]): d = the other
// end's component (the labels of e's original ends are followed through the
// label maps of earlier rounds).  If c and d chose each other (same key) only
// the smaller id acts.  Then: repeat { rc = root(c), rd = root(d); stop if
// equal; CAS parent[max] from max to min }.  Parents always point to smaller
// ids, so the forest never gets a cycle; the thread whose CAS succeeds marks
// e and counts its weight.
__global__ void __launch_bounds__(kBlock) k_hook(int round, const int32_t* __restrict__ src,
                                                 const int32_t* __restrict__ dst,
                                                 const uint32_t* __restrict__ w,
                                                 const unsigned long long* __restrict__ best,
                                                 int32_t* parent, const int32_t* __restrict__ labpool,
                                                 DevState* __restrict__ st,
                                                 uint8_t* __restrict__ in_mst,
                                                 uint32_t* __restrict__ part_sel,
                                                 unsigned long long* __restrict__ part_w) {
  __shared__ uint32_t red32[kWaves];
  __shared__ unsigned long long red64[kWaves];
  const int32_t nr = st->n[round];
  uint32_t sel = 0;
  unsigned long long wsum = 0;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t ci = (int64_t)blockIdx.x * kBlock + threadIdx.x; ci < nr; ci += stride) {
    const int32_t c = (int32_t)ci;
    const unsigned long long key = best[c];
    if (key == kKeyNone) continue;
    const uint32_t e = (uint32_t)key;
    int32_t u = src[e];
    int32_t v = dst[e];
    for (int j = 0; j < round; ++j) {
      const int64_t off = st->lab_off[j];
      u = labpool[off + u];
      v = labpool[off + v];
    }
    const int32_t d = (u == c) ? v : u;
    if ((uint32_t)d >= (uint32_t)nr || (u != c && v != c)) {
      st->err_internal = 1;  // inconsistent labels: never expected, reported as a device error
      continue;
    }
    if (d < c && best[d] == key) continue;  // mutual choice: d hooks it
    int32_t rc = c, rd = d;
    while (true) {
      rc = hook_find(parent, rc);
      rd = hook_find(parent, rd);
      if (rc == rd) break;
      const int32_t hi = rc > rd ? rc : rd;
      const int32_t lo = rc > rd ? rd : rc;
      int32_t expect = hi;
      if (__hip_atomic_compare_exchange_strong(parent + hi, &expect, lo, __ATOMIC_RELAXED,
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
        in_mst[e] = 1;
        ++sel;
        wsum += w[e];
        break;
      }
    }
  }
  sel = block_sum(sel, red32);
  wsum = block_sum(wsum, red64);
  if (threadIdx.x == 0) {
    part_sel[blockIdx.x] = sel;
    part_w[blockIdx.x] = wsum;
  }
}

// ---------------------------------------------------------------- compress

// root_of[c] = root of c (path halving with plain accesses: parent[] only
// changes by halving here, and every value written is an ancestor).  One wave
// handles 64 consecutive components; its ballot of "root with an outgoing
// edge" becomes rootmask[c / 64], its popcount rootcnt[c / 64].  A root
// without a minimum edge is an isolated component: it is final and gets no
// new label.
__global__ void __launch_bounds__(kBlock) k_compress(int round, int32_t* parent,
                                                     int32_t* __restrict__ root_of,
                                                     const unsigned long long* __restrict__ best,
                                                     unsigned long long* __restrict__ rootmask,
                                                     int32_t* __restrict__ rootcnt,
                                                     const DevState* __restrict__ st) {
  const int32_t nr = st->n[round];
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t base = (int64_t)blockIdx.x * kBlock + (threadIdx.x & ~63); base < nr; base += stride) {
    const int64_t ci = base + lane_id();
    bool keep = false;
    if (ci < nr) {
      const int32_t c = (int32_t)ci;
      int32_t cur = c;
      int32_t p = parent[cur];
      while (p != cur) {
        const int32_t gp = parent[p];
        if (gp == p) {
          cur = p;
          break;
        }
        parent[cur] = gp;
        cur = gp;
        p = parent[cur];
      }
      root_of[c] = cur;
      keep = (cur == c) && (best[c] != kKeyNone);
    }
    const uint64_t mask = __ballot(keep);
    if (lane_id() == 0) {
      rootmask[base >> 6] = mask;
      rootcnt[base >> 6] = (int32_t)__popcll(mask);
    }
  }
}

// ---------------------------------------------------------------- finalize

// One workgroup of 1024 threads.  Exclusive scan of rootcnt[0..W) into
// rootpre, W = ceil(n_r / 64); n_{r+1} = total.  Reduces the per-block
// partials of this round: live edges (part_live[0..nlive)), edges added and
// their weight (part_sel / part_w [0..nhook)); adds the weight to *total.
__global__ void __launch_bounds__(1024) k_finalize(int round, const int32_t* __restrict__ rootcnt,
                                                   int32_t* __restrict__ rootpre,
                                                   const uint32_t* __restrict__ part_live, int32_t nlive,
                                                   const uint32_t* __restrict__ part_sel,
                                                   const unsigned long long* __restrict__ part_w,
                                                   int32_t nhook, DevState* st,
                                                   unsigned long long* total) {
  __shared__ int64_t sh[1024 / 64];
  __shared__ unsigned long long shw[1024 / 64];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int32_t nr = st->n[round];
  const int32_t W = (nr + 63) >> 6;
  const int32_t per = (W + 1023) / 1024;
  const int32_t lo = min(W, tid * per), hi = min(W, lo + per);
  int64_t mine = 0;
  for (int32_t i = lo; i < hi; ++i) mine += rootcnt[i];
  // inclusive scan of `mine` across the block
  int64_t x = mine;
  for (int off = 1; off < 64; off <<= 1) {
    const int64_t y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) sh[wv] = x;
  __syncthreads();
  int64_t wave_base = 0, total_roots = 0;
  for (int i = 0; i < 16; ++i) {
    wave_base += (i < wv) ? sh[i] : 0;
    total_roots += sh[i];
  }
  int64_t run = wave_base + x - mine;  // exclusive prefix of this thread's span
  for (int32_t i = lo; i < hi; ++i) {
    rootpre[i] = (int32_t)run;
    run += rootcnt[i];
  }
  // reductions of the partials
  int64_t live = 0, sel = 0;
  unsigned long long ws = 0;
  for (int32_t i = tid; i < nlive; i += 1024) live += part_live[i];
  for (int32_t i = tid; i < nhook; i += 1024) {
    sel += part_sel[i];
    ws += part_w[i];
  }
  live = wave_sum(live);
  sel = wave_sum(sel);
  ws = wave_sum(ws);
  __syncthreads();
  if (lane == 0) {
    sh[wv] = live;
    shw[wv] = ws;
  }
  __syncthreads();
  if (tid == 0) {
    int64_t L = 0;
    unsigned long long S = 0;
    for (int i = 0; i < 16; ++i) {
      L += sh[i];
      S += shw[i];
    }
    st->live[round] = L;
    st->n[round + 1] = (int32_t)total_roots;
    st->lab_off[round + 1] = st->lab_off[round] + nr;
    *total += S;
  }
  __syncthreads();
  if (lane == 0) sh[wv] = sel;
  __syncthreads();
  if (tid == 0) {
    int64_t T = 0;
    for (int i = 0; i < 16; ++i) T += sh[i];
    st->sel[round] = T;
    st->edges_added += T;
  }
}

// ----------------------------------------------------------------- relabel

// lab_r[c] = dense new label of c's root: the number of kept roots with a
// smaller id (rootpre of its 64-word plus a popcount inside the word); -1 for
// an isolated component.  Then parent[] and best[] are reset for the
// n_{r+1} components of the next round.
__global__ void __launch_bounds__(kBlock) k_relabel(int round, const int32_t* __restrict__ root_of,
                                                    const unsigned long long* __restrict__ rootmask,
                                                    const int32_t* __restrict__ rootpre,
                                                    int32_t* __restrict__ labpool, int32_t* parent,
                                                    unsigned long long* best,
                                                    const DevState* __restrict__ st) {
  const int32_t nr = st->n[round];
  const int32_t nn = st->n[round + 1];
  const int64_t off = st->lab_off[round];
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x; c < nr; c += stride) {
    const int32_t r = root_of[c];
    const unsigned long long word = rootmask[r >> 6];
    const int bit = r & 63;
    int32_t label = -1;
    if ((word >> bit) & 1ull) label = rootpre[r >> 6] + __popcll(word & ((1ull << bit) - 1ull));
    labpool[off + c] = label;
  }
  for (int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x; c < nn; c += stride) {
    parent[c] = (int32_t)c;
    best[c] = kKeyNone;
  }
}

// ------------------------------------------------------------ launchers

#define MSTX_LAUNCH_CHECK()                                   \
  do {                                                        \
    hipError_t _e = hipGetLastError();                        \
    if (_e != hipSuccess) return _e;                          \
  } while (0)

hipError_t launch_init(int32_t n, uint32_t m, unsigned long long* best, int32_t* parent, DevState* st,
                       int grid, hipStream_t s) {
  k_init<<<grid, kBlock, 0, s>>>(n, m, best, parent, st);
  MSTX_LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_fill_u64(unsigned long long* p, int64_t count, unsigned long long v, int grid, hipStream_t s) {
  k_fill_u64<<<grid, kBlock, 0, s>>>(p, count, v);
  MSTX_LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_scan_first(bool lds, const int32_t* src, const int32_t* dst, const uint32_t* w, uint32_t m,
                             int32_t n, unsigned long long* best, uint32_t* part_live, DevState* st,
                             int grid, hipStream_t s) {
  if (lds) {
    k_scan_first<true><<<grid, kBlock, (size_t)n * 8, s>>>(src, dst, w, m, n, best, part_live, st);
  } else {
    k_scan_first<false><<<grid, kBlock, 0, s>>>(src, dst, w, m, n, best, part_live, st);
  }
  MSTX_LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_scan_seg(bool from_input, bool lds, int32_t nr_host, int round, const int32_t* src,
                           const int32_t* dst, const uint32_t* w, uint32_t m, const int32_t* labpool,
                           uint4* rec, uint32_t* seg_cnt, uint32_t seg_cap, int32_t nseg,
                           unsigned long long* best, const DevState* st, int grid, hipStream_t s) {
  const size_t sh = lds ? (size_t)nr_host * 8 : 0;
  if (from_input) {
    if (lds)
      k_scan_seg<true, true><<<grid, kBlock, sh, s>>>(round, src, dst, w, m, labpool, rec, seg_cnt, seg_cap, nseg, best, st);
    else
      k_scan_seg<true, false><<<grid, kBlock, 0, s>>>(round, src, dst, w, m, labpool, rec, seg_cnt, seg_cap, nseg, best, st);
  } else {
    if (lds)
      k_scan_seg<false, true><<<grid, kBlock, sh, s>>>(round, src, dst, w, m, labpool, rec, seg_cnt, seg_cap, nseg, best, st);
    else
      k_scan_seg<false, false><<<grid, kBlock, 0, s>>>(round, src, dst, w, m, labpool, rec, seg_cnt, seg_cap, nseg, best, st);
  }
  MSTX_LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_hook(int round, const int32_t* src, const int32_t* dst, const uint32_t* w,
                       const unsigned long long* best, int32_t* parent, const int32_t* labpool,
                       DevState* st, uint8_t* in_mst, uint32_t* part_sel, unsigned long long* part_w,
                       int grid, hipStream_t s) {
  k_hook<<<grid, kBlock, 0, s>>>(round, src, dst, w, best, parent, labpool, st, in_mst, part_sel, part_w);
  MSTX_LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_compress(int round, int32_t* parent, int32_t* root_of, const unsigned long long* best,
                           unsigned long long* rootmask, int32_t* rootcnt, const DevState* st, int grid,
                           hipStream_t s) {
  k_compress<<<grid, kBlock, 0, s>>>(round, parent, root_of, best, rootmask, rootcnt, st);
  MSTX_LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_finalize(int round, const int32_t* rootcnt, int32_t* rootpre, const uint32_t* part_live,
                           int32_t nlive, const uint32_t* part_sel, const unsigned long long* part_w,
                           int32_t nhook, DevState* st, unsigned long long* total, hipStream_t s) {
  k_finalize<<<1, 1024, 0, s>>>(round, rootcnt, rootpre, part_live, nlive, part_sel, part_w, nhook, st, total);
  MSTX_LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_relabel(int round, const int32_t* root_of, const unsigned long long* rootmask,
                          const int32_t* rootpre, int32_t* labpool, int32_t* parent,
                          unsigned long long* best, const DevState* st, int grid, hipStream_t s) {
  k_relabel<<<grid, kBlock, 0, s>>>(round, root_of, rootmask, rootpre, labpool, parent, best, st);
  MSTX_LAUNCH_CHECK();
  return hipSuccess;
}

}  // namespace mstx
