// mstx_kernels.hip -- device kernels of the parallel Boruvka MST for CDNA4 (gfx950).
//
// One Boruvka round (Durbhakula, arXiv 2005.06913, Section 2.1; union and find of
// Section 2.2.2) is a short chain of kernels, each a global barrier for the
// next:
//
//   scan      every live edge: labels of both ends at this round; drop it if
//             internal (the paper's "covered" edge); otherwise offer the
//             packed key (w << 32) | e to the minima of both components --
//             the order is strict, so ties cannot occur (from round 1 on
//             the low half is the record's position in the stream, which
//             orders like e; the hook reads the record there).  From round 1 on
//             the survivors are also compacted in place.  Four ways to
//             take the minima, chosen per round on the device from the
//             actual component count n_r:
//               DENSE   n_r <= kDenseMax: the lightest edge of every
//                       component PAIR in LDS; k_dense_finish then completes
//                       the tree in one workgroup and the round is the last
//                       (any other edge between two components closes a
//                       cycle with a lighter one);
//               LDS     n_r fits one workgroup's LDS: per-workgroup minima
//                       with ds_min_u64, flushed once to HBM;
//               BUCKET  components are split into 256 (at most 1023)
//                       buckets of consecutive components; the scan
//                       counting-sorts its 8-byte offers (weight, slot in
//                       the segment, component in the bucket) by bucket in
//                       LDS and writes them out; k_bucket_min (a workgroup
//                       per bucket, more for a heavy one) takes the minima
//                       in LDS and writes best[];
//               GLOBAL  filtered 64-bit atomicMin on best[] (very large n_r).
//   hook      every component with a minimum: its parent becomes the
//             component at the far end of its lightest edge (the smaller of
//             a mutual pair stays a root); it marks that edge.
//   compress  path halving: every component finds its root; a wave ballot
//             records which roots still have an outgoing edge.
//   finalize  one workgroup: exclusive scan of the root counts (dense new
//             labels), per-round totals, a small record for the host.
//   relabel   old label -> new label map; reset parent[] and the minima.
//   (round tail: when the round has few components, hook .. relabel run in
//   one workgroup with the parent forest in LDS, k_round_tail.  Sparse
//   finish: a late round whose components have few neighbours collects the
//   lightest edge of every component pair into a hash table and, when they
//   fit, ends the solve in one workgroup, k_pair_collect / k_sparse_finish.)
//
// Layout: vertex state is structure-of-arrays in HBM.  The edge stream of
// rounds 0 and 1 is the caller's src/dst/w arrays; from round 2 on it is a
// record stream cut into fixed segments of 4096 records, one segment per
// workgroup iteration, compacted in place: {a, b, w, e} (16 B, one dwordx4),
// or once the labels fit 16 bits a | b << 16 | w << 32 (8 B) with e apart.
//
// Device-scope 64-bit atomics on gfx950 execute at the memory side (~27
// Gop/s whatever the table size) and same-address atomics serialise, so the
// hot paths avoid them: minima live in LDS, per-block partial sums go to
// arrays reduced by the single-workgroup finalize.
//
// Every kernel of round r returns at once when n_r <= 1: the host enqueues
// round r+1 before it has seen the result of round r.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "mstx_internal.h"

namespace mstx {

static constexpr int kBlock = 256;  // threads per workgroup, vertex-parallel kernels
static constexpr int kScanWaves = kScanBlock / 64;

// ------------------------------------------------------------------ helpers

// Streaming accesses (read or written once per round) carry the non-temporal
// hint so they do not evict the label maps and minima that the gathers reuse.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <typename T>
__device__ __forceinline__ T ld_stream(const T* p) {
  return __builtin_nontemporal_load(p);
}
template <typename T>
__device__ __forceinline__ void st_stream(T v, T* p) {
  __builtin_nontemporal_store(v, p);
}
__device__ __forceinline__ uint4 ld_rec(const uint4* p) {
  const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(p));
  return make_uint4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void st_rec(const uint4& r, uint4* p) {
  u32x4 v;
  v.x = r.x;
  v.y = r.y;
  v.z = r.z;
  v.w = r.w;
  __builtin_nontemporal_store(v, reinterpret_cast<u32x4*>(p));
}

__device__ __forceinline__ uint64_t make_key(uint32_t w, uint32_t e) {
  return ((uint64_t)w << 32) | (uint64_t)e;
}

// Lower best[c] to key; the plain load filters the memory-side atomic.  Keys
// only decrease, so a stale load is too large and never skips a needed update.
__device__ __forceinline__ void lower_global(unsigned long long* best, int64_t c, uint64_t key) {
  if (key < best[c]) atomicMin(best + c, (unsigned long long)key);
}

__device__ __forceinline__ void lower_lds(unsigned long long* t, int32_t c, uint64_t key) {
  if (key < t[c]) atomicMin(t + c, (unsigned long long)key);
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// c / g.width for 0 <= c < 2^24: the reciprocal product is at most one too large
__device__ __forceinline__ int32_t bucket_of(int32_t c, const BucketGeom& g) {
  int32_t q = (int32_t)__umulhi((uint32_t)c, g.magic);
  if (q * g.width > c) --q;
  return q;
}

__device__ __forceinline__ uint64_t lanemask_lt() {
  const int l = lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum over the block (NW waves); result valid in every thread.
template <int NW, typename T>
__device__ __forceinline__ T block_sum(T v, T* scratch /* [NW] */) {
  v = wave_sum(v);
  __syncthreads();
  if (lane_id() == 0) scratch[threadIdx.x >> 6] = v;
  __syncthreads();
  T s = 0;
#pragma unroll
  for (int i = 0; i < NW; ++i) s += scratch[i];
  return s;
}


// Copies the n label-map entries at src (labels >= -1) into LDS as label + 1,
// eight loads in flight per thread.
template <typename LabT, int kThreads>
__device__ __forceinline__ void stage_map(LabT* dst, const int32_t* __restrict__ src, int32_t n) {
  for (int32_t i0 = 0; i0 < n; i0 += 8 * kThreads) {
    int32_t v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int32_t i = i0 + q * kThreads + (int32_t)threadIdx.x;
      v[q] = src[i < n ? i : 0];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int32_t i = i0 + q * kThreads + (int32_t)threadIdx.x;
      if (i < n) dst[i] = (LabT)(v[q] + 1);
    }
  }
}

// --------------------------------------------------------------------- init

// best[0..n) <- none, parent[c] <- c, state for round 0.
__global__ void __launch_bounds__(kBlock) k_init(int32_t n, int64_t m, int64_t cmap_off, int dense_limit,
                                                 unsigned long long* best, int32_t* parent,
                                                 unsigned long long* pbest, uint32_t* btot, SparseTable sp,
                                                 DevState* st) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  if (sp.pid) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < kSparseHash; i += stride) {
      sp.pid[i] = kPairEmpty;
      sp.key[i] = kKeyNone;
    }
    if (blockIdx.x == 0 && threadIdx.x < 2) sp.state[threadIdx.x] = 0;
  }
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += stride) {
    best[c] = kKeyNone;
    parent[c] = (int32_t)c;
  }
  if (pbest)
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < kDensePairsMax; i += stride)
      pbest[i] = kKeyNone;
  if (btot)
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < kMaxBuckets; i += stride) btot[i] = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->n[0] = n;
    st->lab_off[0] = 0;
    st->m = m;
    st->stream[0] = m;
    st->map_off[0] = 0;
    st->map_n[0] = 0;
    st->keep[0] = 0;
    st->cmap_off = cmap_off;
    st->dense_limit = dense_limit;
    st->err = 0;
    st->err_internal = 0;
    st->edges_added = 0;
    st->dense_at = -1;
  }
}

// p[0 .. count) = v, bytes (a kernel rather than a memset node, so that a
// captured graph clears the flags with a kernel).
__global__ void __launch_bounds__(kBlock) k_fill_u8(uint8_t* p, int64_t count, uint8_t v) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < count; i += stride) p[i] = v;
}

__global__ void __launch_bounds__(kBlock) k_fill_u64(unsigned long long* p, int64_t count, unsigned long long v) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) p[i] = v;
}

// --------------------------------------------------------------------- scan

// One kernel for every round and mode.  kStage is the edge stream the round
// reads (scan_stage):
//   0  round 0: the caller's edges, labels = vertex ids, ids checked against
//      [0, n) (st->err on failure); nothing is compacted
//   1  round 1: the caller's edges, labels through round 0's map
//   2  wide records {a, b, w, e} of an earlier round, labels through the map
//      of this round (map_off / map_n)
//   3  narrow records (a | b << 16 | w << 32, e apart), the same way
// From round 1 on the survivors are rewritten in place (narrow when this
// round's labels fit 16 bits), unless the round keeps its narrow records
// where they are (st->keep) or is a dense round (its round is the last).
// kMode is the way minima are taken (LDS / BUCKET / GLOBAL / DENSE); a launch
// whose mode is not the one pick_mode() selects for the actual n_r returns.
// Dynamic LDS: LDS mode n_r (<= launch capacity) u64 minima; DENSE mode
// n_r (n_r - 1) / 2 u64 pair minima; BUCKET mode the 2 * kSegCap offer staging
// and the (bucket count + 1) counters.
template <int kMode, int kStage>
__global__ void __launch_bounds__(kScanBlock) k_scan(ScanArgs A) {
  constexpr bool kFromInput = kStage <= 1;
  constexpr bool kCompact = kStage >= 1;  // labels come through a map; survivors may be rewritten
  constexpr bool kNarrowIn = kStage == 3;
  // round 1 reads the caller's edges again: the ones round 0 added join two
  // vertices of one component, so they are dead without their label lookups
  const bool skip_added = kStage == 1 && A.in_mst != nullptr;
  extern __shared__ unsigned long long smem[];
  __shared__ uint32_t slot_tot[kPerThread * kScanWaves];  // survivors per (slot k, wave)
  __shared__ uint32_t red[kScanWaves];
  static_assert(kPerThread * kScanWaves == 64, "one lane per (slot, wave) pair");
  const int32_t nr = A.st->n[A.round];
  if (nr <= 1 && A.round > 0) return;
  // a round enqueued before the host saw an input error in round 0 does nothing
  if (A.round > 0 && A.st->err) return;
  if (pick_mode(nr, A.launched) != kMode) return;
  const int32_t* lab = kCompact ? A.labpool + A.st->map_off[A.round] : nullptr;
  // this round's survivors: rewritten (moved to their compacted positions),
  // narrow or wide, left where they are, or relabelled where they are
  const int what = kNarrowIn ? A.st->keep[A.round] : kMoveRecords;
  const bool moved = kCompact && kMode != kModeDense && what == kMoveRecords;
  const bool inplace = kNarrowIn && kMode != kModeDense && what == kRelabelRecords;
  const bool narrow_out = nr <= kNarrowMax;
  // keys carry stream positions from round 1 on (see below)
  constexpr bool kPosKey = kCompact && !(kFromInput && kMode == kModeDense);
  // rounds >= 2 in LDS / DENSE mode: the first entries of this round's label
  // map are staged in LDS behind the minima table for the actual n_r, as
  // many as the launch's allocation holds.  Its values are labels of this
  // round, below n_r, or -1 (isolated): they are stored plus one in 2 bytes
  // (LDS mode, n_r <= kLdsSlots) or 1 byte (DENSE mode, n_r <= kDenseMax).
  // Lookups: 0 the vertex ids themselves (round 0), 1 the map in memory,
  // 2 LDS for every label, 3 LDS below the staged count and memory above.
  using LabT = std::conditional_t<kMode == kModeDense, uint8_t, uint16_t>;
  static_assert(kLdsSlots < 0xFFFF && kDenseMax < 0xFF, "staged labels plus one fit their type");
  const LabT* llab = nullptr;
  int lookup = kCompact ? 1 : 0;
  int32_t nst = 0;
  if (!kFromInput && (kMode == kModeLds || kMode == kModeDense)) {
    const int32_t table = kMode == kModeDense ? dense_pairs(nr) * 8 : nr * 8;
    const int32_t off = (table + 15) & ~15;
    const int32_t room = (A.lds_bytes - off) / (int32_t)sizeof(LabT);
    const int32_t nmap = A.st->map_n[A.round];
    nst = room <= 0 ? 0 : (nmap < room ? nmap : room);
    if (nst > 0) {
      LabT* dst_l = reinterpret_cast<LabT*>(reinterpret_cast<char*>(smem) + off);
      stage_map<LabT, kScanBlock>(dst_l, lab, nst);
      llab = dst_l;  // visible to all after the table initialisation's barrier below
      lookup = nst == nmap ? 2 : 3;
    }
  }

  unsigned long long* lbest = smem;  // LDS mode
  // BUCKET mode: geometry derived from n_r exactly as k_bucket_min does
  BucketGeom bg{1, 0, 0};
  int nbk = 0;
  uint32_t* bcnt = nullptr;
  unsigned long long* soff = nullptr;
  if (kMode == kModeBucket) {
    bg = bucket_geometry(nr);
    nbk = bg.nbk;
    soff = smem;                                           // [kOfferCap]
    bcnt = reinterpret_cast<uint32_t*>(soff + kOfferCap);  // [nbk + 1]
  }
  if (kMode == kModeLds) {
    for (int32_t c = threadIdx.x; c < nr; c += kScanBlock) lbest[c] = kKeyNone;
    __syncthreads();
  }
  const int32_t npairs = kMode == kModeDense ? dense_pairs(nr) : 0;
  if (kMode == kModeDense) {
    for (int32_t c = threadIdx.x; c < npairs; c += kScanBlock) lbest[c] = kKeyNone;
    __syncthreads();
  }
  const int wave = threadIdx.x >> 6;
  const uint64_t lt = lanemask_lt();
  bool bad = false;
  uint32_t my_btot = 0;  // BUCKET mode: offers of bucket threadIdx.x in this workgroup's segments
  const unsigned long long* nrec_in = reinterpret_cast<const unsigned long long*>(A.rec);
  const uint32_t* ne_in = reinterpret_cast<const uint32_t*>(A.rec);

  // Raw loads of a segment: (src, dst, w, e) from the caller's arrays, the
  // wide record (a, b, w, e), or the narrow record (a | b << 16, -, w, e) of
  // an earlier round (e only when the round moves its survivors; loaded
  // first, so that the wait for the record words also covers it: vector
  // memory loads complete in issue order).  The next segment of this
  // workgroup is loaded while the current one is processed (its loads stay
  // in flight across the barriers, which wait for LDS only).
  auto seg_count = [&](int32_t s) -> uint32_t {
    const uint64_t base = (uint64_t)s * kSegCap;
    if (kFromInput) return base >= A.m ? 0u : (uint32_t)min((uint64_t)kSegCap, (uint64_t)A.m - base);
    return A.seg_cnt[s];
  };
  // Record loads are unconditional (lanes past the segment's count read its
  // first slot, in bounds, and are masked later) so that no branch makes the
  // compiler wait for them early.  A record segment's count is loaded two
  // segments ahead, so it has arrived when that segment's loads are issued.
  auto load_seg = [&](int32_t s, uint32_t count, uint4* x, uint32_t* added) {
    const uint64_t base = (uint64_t)s * kSegCap;
    if (kNarrowIn) {
      // this segment's narrow records and their edge indices (narrow_rec_index, narrow_e_index)
      const unsigned long long* nseg = nrec_in + 2 * base;
      const uint32_t* eseg = ne_in + 4 * base + 2 * kSegCap;
      uint32_t ev[kPerThread];
#pragma unroll
      for (int k = 0; k < kPerThread; ++k) {
        const uint32_t j = k * kScanBlock + threadIdx.x;
        ev[k] = moved ? ld_stream(eseg + (j < count ? j : 0u)) : 0u;
      }
      __asm__ __volatile__("" ::: "memory");  // the e loads are issued before the record loads
#pragma unroll
      for (int k = 0; k < kPerThread; ++k) {
        const uint32_t j = k * kScanBlock + threadIdx.x;
        const unsigned long long v = ld_stream(nseg + (j < count ? j : 0u));
        x[k] = make_uint4((uint32_t)v, 0u, (uint32_t)(v >> 32), ev[k]);
      }
      return;
    }
    uint32_t bits = 0;
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) {
      const uint32_t j = k * kScanBlock + threadIdx.x;
      if (kFromInput) {
        x[k] = make_uint4(0, 0, 0, 0);
        if (j < count) {
          const uint32_t e = (uint32_t)(base + j);
          x[k] = make_uint4((uint32_t)ld_stream(A.src + e), (uint32_t)ld_stream(A.dst + e), ld_stream(A.w + e), e);
          // round 1: bit k when round 0 added the edge.  Taking the bits here
          // waits for this segment's loads (they were issued last), so the
          // current segment's label lookups, which come next, find no
          // streaming load in flight beside them: measured faster on the
          // random and R-MAT graphs than reading the flags later.
          if (skip_added && ld_stream(A.in_mst + e)) bits |= 1u << k;
        }
      } else {
        x[k] = ld_rec(A.rec + base + (j < count ? j : 0u));
      }
    }
    *added = bits;
  };
  uint4 nx[kPerThread];
  uint32_t nadded = 0;
  uint32_t ncount = 0, nncount = 0;
  if ((int32_t)blockIdx.x < A.nseg) {
    ncount = seg_count(blockIdx.x);
    if (!kFromInput && (int32_t)(blockIdx.x + gridDim.x) < A.nseg) nncount = seg_count(blockIdx.x + gridDim.x);
    load_seg(blockIdx.x, ncount, nx, &nadded);
  }
  for (int32_t s = blockIdx.x; s < A.nseg; s += gridDim.x) {
    const uint64_t base = (uint64_t)s * kSegCap;
    const uint32_t count = ncount;
    // the next segment of this workgroup; for the record stream, after the
    // last one the current segment is loaded again (cache hits), so the loads
    // are issued on every path and the compiler's wait counts stay exact
    const bool has_next = s + (int32_t)gridDim.x < A.nseg;
    const int32_t sn = has_next ? s + (int32_t)gridDim.x : s;
    uint4 cx[kPerThread];
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) cx[k] = nx[k];
    const uint32_t cadded = nadded;
    // Vector-memory counters retire in issue order.  The next segment's
    // count goes first.  From the caller's arrays the next segment's loads
    // follow (round 1's label lookups miss to the last-level cache anyway);
    // from the record stream this segment's label lookups go first, so they
    // complete while the next records are still in flight.
    if (kFromInput) {
      if (has_next) {
        ncount = seg_count(sn);
        load_seg(sn, ncount, nx, &nadded);
      }
    } else {
      // the next segment's count arrived during the last segment; the one
      // after it is loaded now
      ncount = has_next ? nncount : count;
      const int64_t snn = (int64_t)s + 2 * (int64_t)gridDim.x;
      nncount = snn < A.nseg ? seg_count((int32_t)snn) : 0u;
    }
    __asm__ __volatile__("" ::: "memory");
    // this round's labels of both ends (lanes past the count look up entry 0)
    int32_t ga[kPerThread], gb[kPerThread];
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) {
      const bool in = k * kScanBlock + threadIdx.x < count;
      ga[k] = in ? (int32_t)(kNarrowIn ? cx[k].x & 0xFFFFu : cx[k].x) : 0;
      gb[k] = in ? (int32_t)(kNarrowIn ? cx[k].x >> 16 : cx[k].y) : 0;
    }
    if (kFromInput && !kCompact) {
#pragma unroll
      for (int k = 0; k < kPerThread; ++k) {
        if ((uint32_t)ga[k] >= (uint32_t)A.n || (uint32_t)gb[k] >= (uint32_t)A.n) {
          bad = true;
          ga[k] = gb[k] = -1;  // dropped
        }
      }
    } else if (lookup == 2) {
#pragma unroll
      for (int k = 0; k < kPerThread; ++k) {
        ga[k] = (int32_t)llab[ga[k]] - 1;
        gb[k] = (int32_t)llab[gb[k]] - 1;
      }
    } else if (lookup == 3) {
#pragma unroll
      for (int k = 0; k < kPerThread; ++k) {
        ga[k] = ga[k] < nst ? (int32_t)llab[ga[k]] - 1 : lab[ga[k]];
        gb[k] = gb[k] < nst ? (int32_t)llab[gb[k]] - 1 : lab[gb[k]];
      }
    } else {
#pragma unroll
      for (int k = 0; k < kPerThread; ++k) {
        if ((cadded >> k) & 1u) {
          ga[k] = gb[k] = -1;  // added in round 0: both ends in one component, dead
        } else {
          ga[k] = lab[ga[k]];
          gb[k] = lab[gb[k]];
        }
      }
    }
    __asm__ __volatile__("" ::: "memory");
    if (!kFromInput) load_seg(sn, ncount, nx, &nadded);
    __asm__ __volatile__("" ::: "memory");
    if (kMode == kModeBucket) {
      for (int i = threadIdx.x; i <= nbk; i += kScanBlock) bcnt[i] = 0;
      __syncthreads();
    }
    uint4 r[kPerThread];
    bool live[kPerThread];
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) {
      const uint32_t j = k * kScanBlock + threadIdx.x;
      live[k] = false;
      r[k] = make_uint4(0, 0, 0, 0);
      if (j < count) {
        const int32_t a = ga[k], b = gb[k];
        const uint32_t we = cx[k].z, e = cx[k].w;
        r[k] = make_uint4((uint32_t)a, (uint32_t)b, we, e);
        // a live edge never touches an isolated (label -1) component
        live[k] = (a != b) && ((a | b) >= 0);
      }
    }

    // survivors of this segment, in input order: record j = k * kScanBlock +
    // threadIdx.x, so the order is (slot k, wave, lane); rank inside the
    // wave's slot now, offsets of the (k, wave) groups after the barrier
    // (ranks only when the survivors move)
    uint32_t my_off[kPerThread];
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) {
      const uint64_t mask = __ballot(live[k]);
      my_off[k] = moved ? (uint32_t)__popcll(mask & lt) : 0u;
      if (lane_id() == 0) slot_tot[k * kScanWaves + wave] = (uint32_t)__popcll(mask);
    }

    // BUCKET mode: claim a slot in the offer staging for both ends
    // (slot in its bucket's run in bits 0..15, the bucket in bits 16..)
    uint32_t slot_a[kPerThread], slot_b[kPerThread];
    if (kMode == kModeBucket) {
#pragma unroll
      for (int k = 0; k < kPerThread; ++k) {
        slot_a[k] = slot_b[k] = 0;
        if (live[k]) {
          const uint32_t qa = (uint32_t)bucket_of((int32_t)r[k].x, bg);
          const uint32_t qb = (uint32_t)bucket_of((int32_t)r[k].y, bg);
          slot_a[k] = atomicAdd(&bcnt[qa], 1u) | (qa << 16);
          slot_b[k] = atomicAdd(&bcnt[qb], 1u) | (qb << 16);
        }
      }
    }
    __syncthreads();  // all reads of this segment are done past this point

    uint32_t seg_tot;
    {
      // exclusive scan of the 64 group counts across one wave's lanes
      const uint32_t v = slot_tot[lane_id()];
      uint32_t x = v;
      for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off, 64);
        if (lane_id() >= off) x += y;
      }
      seg_tot = __shfl(x, 63, 64);
      const uint32_t excl = x - v;
      if (moved) {
#pragma unroll
        for (int k = 0; k < kPerThread; ++k) my_off[k] += __shfl(excl, k * kScanWaves + wave, 64);
      }
    }
    // Keys: the weight in the high half; in the low half the edge's index
    // (round 0, and a dense round that reads the caller's arrays) or the
    // edge's position in the record stream after this scan.  The stream keeps
    // the input order (stable compaction inside fixed segments), so
    // positions break ties exactly as indices do, and the hook reads the
    // record there (the labels and the edge index) instead of following the
    // label maps of every earlier round.  A round that moves no record (dense,
    // or keeping its records) keys the positions it read.
    uint64_t key[kPerThread];
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) {
      const uint32_t j = k * kScanBlock + threadIdx.x;
      const uint32_t pos = moved ? (uint32_t)(base + my_off[k]) : (uint32_t)(base + j);
      key[k] = make_key(r[k].z, kPosKey ? pos : r[k].w);
      if (live[k]) {
        const int32_t a = (int32_t)r[k].x, b = (int32_t)r[k].y;
        if (kMode == kModeDense) {
          const int32_t lo = a < b ? a : b, hi = a < b ? b : a;
          lower_lds(lbest, pair_index(lo, hi, nr), key[k]);
        } else if (kMode == kModeLds) {
          lower_lds(lbest, a, key[k]);
          lower_lds(lbest, b, key[k]);
        } else if (kMode == kModeGlobal) {
          lower_global(A.best, a, key[k]);
          lower_global(A.best, b, key[k]);
        }
      }
    }
    if (inplace) {
      // every record keeps its position and gets this round's labels (an
      // internal one gets labels 0, 0: internal again in every later round)
      unsigned long long* nrec_out = reinterpret_cast<unsigned long long*>(A.rec) + 2 * base;
#pragma unroll
      for (int k = 0; k < kPerThread; ++k) {
        const uint32_t j = k * kScanBlock + threadIdx.x;
        if (j < count) {
          const unsigned long long lb = live[k] ? (unsigned long long)(r[k].x | (r[k].y << 16)) : 0ull;
          st_stream(lb | ((unsigned long long)r[k].z << 32), nrec_out + j);
        }
      }
    }
    if (moved) {
      if (narrow_out) {
        // this segment's narrow records and their edge indices (narrow_rec_index, narrow_e_index)
        unsigned long long* nrec_out = reinterpret_cast<unsigned long long*>(A.rec) + 2 * base;
        uint32_t* ne_out = reinterpret_cast<uint32_t*>(A.rec) + 4 * base + 2 * kSegCap;
#pragma unroll
        for (int k = 0; k < kPerThread; ++k) {
          if (live[k]) {
            st_stream((unsigned long long)(r[k].x | (r[k].y << 16)) | ((unsigned long long)r[k].z << 32),
                      nrec_out + my_off[k]);
            st_stream(r[k].w, ne_out + my_off[k]);
          }
        }
      } else {
#pragma unroll
        for (int k = 0; k < kPerThread; ++k) {
          if (live[k]) st_rec(r[k], A.rec + base + my_off[k]);
        }
      }
    }
    if (kFromInput && !kCompact && kMode != kModeDense) {
      // round 0: src ^ dst of every edge, in the (still unused) record
      // buffer, so the hook finds the other end of a vertex's edge with one
      // 4-byte read
      uint32_t* xends = reinterpret_cast<uint32_t*>(A.rec);
#pragma unroll
      for (int k = 0; k < kPerThread; ++k) {
        const uint32_t j = k * kScanBlock + threadIdx.x;
        if (j < count) st_stream(cx[k].x ^ cx[k].y, xends + base + j);
      }
    }
    if (threadIdx.x == 0) {
      A.seg_live[s] = seg_tot;
      if (moved) A.seg_cnt[s] = seg_tot;
    }

    if (kMode == kModeBucket) {
      // exclusive scan of the (padded) bucket counts (nbk + 1 <= kScanBlock)
      const uint32_t cnt = (int)threadIdx.x < nbk ? bcnt[threadIdx.x] : 0u;
      my_btot += cnt;
      const uint32_t v = nbk <= kOfferPadBuckets ? (cnt + kOfferAlign - 1) & ~(uint32_t)(kOfferAlign - 1) : cnt;
      uint32_t x = v;
      for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off, 64);
        if (lane_id() >= off) x += y;
      }
      if (lane_id() == 63) red[wave] = x;
      __syncthreads();
      uint32_t wbase = 0;
      for (int i = 0; i < wave; ++i) wbase += red[i];
      const uint32_t excl = wbase + x - v;
      __syncthreads();  // every thread has read its counter
      if ((int)threadIdx.x <= nbk) bcnt[threadIdx.x] = excl;  // for threadIdx == nbk this is the total
      if ((int)threadIdx.x < nbk) A.offT[(int64_t)threadIdx.x * A.nseg + s] = excl | (cnt << 16);
      __syncthreads();
#pragma unroll
      for (int k = 0; k < kPerThread; ++k) {
        if (live[k]) {
          const int32_t a = (int32_t)r[k].x, b = (int32_t)r[k].y;
          const int32_t qa = (int32_t)(slot_a[k] >> 16), qb = (int32_t)(slot_b[k] >> 16);
          const uint32_t pa = bcnt[qa] + (slot_a[k] & 0xFFFFu);
          const uint32_t pb = bcnt[qb] + (slot_b[k] & 0xFFFFu);
          // the key's low half is this segment's first position plus the slot
          const uint64_t o = (key[k] & 0xFFFFFFFF00000000ull) |
                             ((uint64_t)((uint32_t)key[k] - (uint32_t)base) << kOfferSlotShift);
          soff[pa] = o | (uint32_t)(a - qa * bg.width);
          soff[pb] = o | (uint32_t)(b - qb * bg.width);
        }
      }
      __syncthreads();
      const uint32_t total = bcnt[nbk];  // offers + pads
      const uint64_t obase = (uint64_t)s * kOfferCap;
      for (uint32_t i = threadIdx.x; i < total; i += kScanBlock) st_stream(soff[i], A.offers + obase + i);
    }
    __syncthreads();  // LDS (group counts, counters, staging) is reused by the next segment
  }
  if (!kCompact && bad) A.st->err = 1;
  if (kMode == kModeBucket && my_btot) atomicAdd(A.btot + threadIdx.x, my_btot);
  if (kMode == kModeDense) {
    __syncthreads();
    if (use_slab(A.slab, A.slab_cap, npairs, gridDim.x, kSlabAnyStream)) {
      unsigned long long* row = A.slab + (int64_t)blockIdx.x * npairs;
      for (int32_t c = threadIdx.x; c < npairs; c += kScanBlock) row[c] = lbest[c];
    } else {
      for (int32_t c = threadIdx.x; c < npairs; c += kScanBlock) {
        const unsigned long long v = lbest[c];
        if (v != kKeyNone) lower_global(A.pbest, c, v);
      }
    }
  }
  if (kMode == kModeLds) {
    __syncthreads();
    if (use_slab(A.slab, A.slab_cap, nr, gridDim.x, A.st->stream[A.round])) {
      // coalesced copy of this workgroup's minima; k_slab_min takes the column minima
      unsigned long long* row = A.slab + (int64_t)blockIdx.x * nr;
      for (int32_t c = threadIdx.x; c < nr; c += kScanBlock) row[c] = lbest[c];
    } else {
      for (int32_t c = threadIdx.x; c < nr; c += kScanBlock) {
        const unsigned long long v = lbest[c];
        if (v != kKeyNone) lower_global(A.best, c, v);
      }
    }
  }
}

// best[c] = min over the nwg workgroup rows of the slab (LDS mode with more
// than kSlabMin components; the scan that wrote the slab had nwg workgroups).
// In dense mode the columns are the component pairs and the target is the
// pair table pbest[].  Block (x, y): columns x*256.., rows
// y*kSlabRowsPerBlock..; each partial minimum is merged with a filtered
// atomicMin (the target was reset to "none").
static constexpr int kSlabRowsPerBlock = 32;
__global__ void __launch_bounds__(kBlock) k_slab_min(int round, int launched, int mode,
                                                     const unsigned long long* __restrict__ slab,
                                                     int64_t slab_cap, int nwg,
                                                     unsigned long long* __restrict__ best,
                                                     unsigned long long* __restrict__ pbest,
                                                     const DevState* __restrict__ st) {
  int32_t nr = st->n[round];
  if (nr <= 1 && round > 0) return;
  if (round > 0 && st->err) return;
  // runs after the scan of `mode` (LDS or dense) and only if that scan ran
  if (pick_mode(nr, launched) != mode) return;
  int64_t stream = st->stream[round];
  if (mode == kModeDense) {
    // columns are the component pairs, the target the pair minima
    nr = dense_pairs(nr);
    best = pbest;
    stream = kSlabAnyStream;
  }
  if (!use_slab(slab, slab_cap, nr, nwg, stream)) return;
  const int b0 = blockIdx.y * kSlabRowsPerBlock;
  const int b1 = min(nwg, b0 + kSlabRowsPerBlock);
  for (int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x; c < nr; c += (int64_t)gridDim.x * kBlock) {
    unsigned long long v = kKeyNone;
    int b = b0;
    for (; b + 8 <= b1; b += 8) {
      unsigned long long x[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) x[u] = slab[(int64_t)(b + u) * nr + c];
#pragma unroll
      for (int u = 0; u < 8; ++u) v = min(v, x[u]);
    }
    for (; b < b1; ++b) v = min(v, slab[(int64_t)b * nr + c]);
    if (v != kKeyNone) lower_global(best, c, v);
  }
}

// Exclusive prefix sum of one value per thread over a 1024-thread block;
// *total receives the sum.  `sh` holds kScanWaves words.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* sh, uint32_t* total) {
  uint32_t x = v;
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(x, off, 64);
    if (lane_id() >= off) x += y;
  }
  const int wv = threadIdx.x >> 6;
  if (lane_id() == 63) sh[wv] = x;
  __syncthreads();
  uint32_t base = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < kScanWaves; ++i) {
    const uint32_t t = sh[i];
    base += i < wv ? t : 0u;
    tot += t;
  }
  __syncthreads();  // sh may be reused
  *total = tot;
  return base + x - v;
}

// Sum of one 64-bit value per thread over a 1024-thread block, returned to
// every thread.  `sh` holds kScanWaves words.
__device__ __forceinline__ unsigned long long block_sum64(unsigned long long v, unsigned long long* sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if (lane_id() == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  unsigned long long tot = 0;
#pragma unroll
  for (int i = 0; i < kScanWaves; ++i) tot += sh[i];
  __syncthreads();  // sh may be reused
  return tot;
}

// The minimum offer of every component of a bucket, over the run
// offT[p][s] (start, length) of the bucket in every segment s, taken in LDS.
//
// Work units: every bucket gets one workgroup, and a bucket with more than
// twice the average number of offers (`btot`, counted by the scan: a hub of
// a skewed graph) gets more, each taking an equal share of the segments;
// the extra workgroups of a launch beyond the units return.  A bucket with
// one unit writes its minima into best[] (reset to "none" for the round); a
// bucket with several merges them with filtered atomics.
//
// Inside a workgroup the runs of a chunk of segments are cut into items of
// at most kItemOffers offers (a run can be long when the edge order has
// locality, e.g. a grid), and half-waves take kRunsInFlight items at a time,
// each read with coalesced loads.
static constexpr int kChunkRuns = 2048;
static constexpr int kRunsInFlight = 8;
static constexpr uint32_t kItemOffers = 128;
// LDS behind the minima table: run words, item prefix, unit prefix
static constexpr size_t kBucketMinExtraLds = (2 * kChunkRuns + 1 + kMaxBuckets + 1) * sizeof(uint32_t);
static_assert(kChunkRuns == 2 * kScanBlock, "two runs per thread in the item scan");

__global__ void __launch_bounds__(kScanBlock) k_bucket_min(int round, int launched,
                                                           const unsigned long long* __restrict__ offers,
                                                           const uint32_t* __restrict__ offT, int32_t nseg,
                                                           const uint32_t* __restrict__ btot,
                                                           unsigned long long* __restrict__ best,
                                                           const DevState* __restrict__ st) {
  extern __shared__ unsigned long long table[];  // [B] minima, then the staging below
  __shared__ uint32_t sh[kScanWaves];
  __shared__ unsigned long long sh64[kScanWaves];
  const int32_t nr = st->n[round];
  if (nr <= 1 && round > 0) return;
  if (round > 0 && st->err) return;  // the scan of this round did nothing either
  if (pick_mode(nr, launched) != kModeBucket) return;
  const BucketGeom bg = bucket_geometry(nr);
  const int nbk = bg.nbk;
  const int B = bg.width;
  uint32_t* run_w = reinterpret_cast<uint32_t*>(table + B);  // [kChunkRuns]
  uint32_t* iprefix = run_w + kChunkRuns;                    // [kChunkRuns + 1]
  uint32_t* uprefix = iprefix + kChunkRuns + 1;              // [kMaxBuckets + 1]
  const int tid = threadIdx.x;

  // work units of every bucket (nbk <= kScanBlock - 1: one bucket per thread);
  // their sum in 64 bits: a round of more than 2^31 live edges makes more
  // than 2^32 offers.  (A single bucket's 32-bit count wraps only past 2^32
  // offers into one bucket; its units are then fewer than they should be,
  // never its segments.)
  const unsigned long long tot_p = tid < nbk ? btot[tid] : 0ull;
  const unsigned long long all = block_sum64(tot_p, sh64);
  // target >= twice the average, so the extra units number at most nbk / 2
  const uint64_t target = max((uint64_t)1, (2 * (uint64_t)all + (uint32_t)nbk - 1) / (uint32_t)nbk);
  uint32_t units = tid < nbk ? 1u + (uint32_t)(tot_p / target) : 0u;
  uint32_t total_units;
  uint32_t ex = block_excl_scan(units, sh, &total_units);
  if (total_units > gridDim.x) {  // never with the host's grid; one unit per bucket then
    ex = (uint32_t)tid;
    total_units = (uint32_t)nbk;
  }
  if (tid < nbk) uprefix[tid] = ex;
  if (tid == 0) uprefix[nbk] = total_units;
  __syncthreads();
  const uint32_t b = blockIdx.x;
  if (b >= total_units) return;
  int lo = 0, hi = nbk;  // uprefix[lo] <= b < uprefix[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (uprefix[mid] <= b) lo = mid;
    else hi = mid;
  }
  const int p = lo;
  const uint32_t U = uprefix[p + 1] - uprefix[p], u = b - uprefix[p];
  const int32_t s_begin = (int32_t)((int64_t)nseg * u / U), s_end = (int32_t)((int64_t)nseg * (u + 1) / U);

  for (int i = tid; i < B; i += kScanBlock) table[i] = kKeyNone;
  const uint32_t* row = offT + (int64_t)p * nseg;
  const int half = tid >> 5;  // 0 .. 2 * kScanWaves - 1
  const int hl = tid & 31;
  constexpr int kHalves = 2 * kScanWaves;
  for (int32_t c0 = s_begin; c0 < s_end; c0 += kChunkRuns) {
    const int nrun = min(kChunkRuns, s_end - c0);
    __syncthreads();  // table initialised / previous chunk's staging consumed
    // runs 2 tid and 2 tid + 1, and their item counts
    const uint32_t w0 = 2 * tid < nrun ? row[c0 + 2 * tid] : 0u;
    const uint32_t w1 = 2 * tid + 1 < nrun ? row[c0 + 2 * tid + 1] : 0u;
    const uint32_t n0 = ((w0 >> 16) + kItemOffers - 1) / kItemOffers;
    const uint32_t n1 = ((w1 >> 16) + kItemOffers - 1) / kItemOffers;
    uint32_t nitems;
    const uint32_t e0 = block_excl_scan(n0 + n1, sh, &nitems);
    run_w[2 * tid] = w0;
    run_w[2 * tid + 1] = w1;
    iprefix[2 * tid] = e0;
    iprefix[2 * tid + 1] = e0 + n0;
    if (tid == 0) iprefix[nrun] = nitems;
    // runs of at most one item (the common case) are taken directly, one per
    // item slot, without the search for a long run's pieces
    const bool short_runs = !__syncthreads_or(n0 > 1 || n1 > 1);
    const uint32_t nslots = short_runs ? (uint32_t)nrun : nitems;
    for (uint32_t i0 = half * kRunsInFlight; i0 < nslots; i0 += kHalves * kRunsInFlight) {
      uint32_t seg[kRunsInFlight], at0[kRunsInFlight], len[kRunsInFlight];
      uint32_t maxlen = 0;
#pragma unroll
      for (int q = 0; q < kRunsInFlight; ++q) {
        seg[q] = 0;
        at0[q] = 0;
        len[q] = 0;
        const uint32_t it = i0 + q;
        if (it < nslots) {
          int rl = (int)it;  // short runs: item it is run it
          uint32_t piece = 0;
          if (!short_runs) {
            int rh = nrun;  // iprefix[rl] <= it < iprefix[rh]
            rl = 0;
            while (rh - rl > 1) {
              const int mid = (rl + rh) >> 1;
              if (iprefix[mid] <= it) rl = mid;
              else rh = mid;
            }
            piece = (it - iprefix[rl]) * kItemOffers;
          }
          const uint32_t wd = run_w[rl];
          seg[q] = (uint32_t)(c0 + rl);
          at0[q] = (wd & 0xFFFFu) + piece;
          len[q] = min(kItemOffers, (wd >> 16) - piece);
        }
        maxlen = max(maxlen, len[q]);
      }
      for (uint32_t i = hl; i < maxlen; i += 32) {
        unsigned long long o[kRunsInFlight];
#pragma unroll
        for (int q = 0; q < kRunsInFlight; ++q) {
          o[q] = 0;
          if (i < len[q]) o[q] = ld_stream(offers + (uint64_t)seg[q] * kOfferCap + at0[q] + i);
        }
#pragma unroll
        for (int q = 0; q < kRunsInFlight; ++q) {
          if (i < len[q]) {
            // the key: weight, and the segment's first position plus the slot
            const uint32_t lo = seg[q] * (uint32_t)kSegCap +
                                (uint32_t)((o[q] >> kOfferSlotShift) & (uint64_t)(kSegCap - 1));
            lower_lds(table, (int32_t)(o[q] & ((1u << kOfferSlotShift) - 1)),
                      (o[q] & 0xFFFFFFFF00000000ull) | lo);
          }
        }
      }
    }
  }
  __syncthreads();
  const int64_t base = (int64_t)p * B;
  for (int i = tid; i < B; i += kScanBlock) {
    const unsigned long long v = table[i];
    if (base + i < nr && v != kKeyNone) {
      if (U == 1) best[base + i] = v;
      else lower_global(best, base + i, v);
    }
  }
}

// ------------------------------------------------------------ dense finish

static constexpr int kDenseThreads = 1024;
static constexpr int kDenseWaves = kDenseThreads / 64;
// Rows of the small graph are scanned by groups of adjacent lanes.
static constexpr int kDenseRowThreads = 4;
static_assert(kDenseMax * kDenseRowThreads <= kDenseThreads, "one lane group per row");
static_assert(kDenseMax <= 256, "the new ids of one round are ranked by one wave");
// The pair table is loaded two keys at a time, all loads issued first.
static constexpr int kDenseLoadIters = (kDensePairsMax / 2 + kDenseThreads - 1) / kDenseThreads;
// A contracted table has at most k/2 vertices, so a quarter of the entries:
// the old entries under it, per thread.
static constexpr int kDenseTopQ = (dense_pairs(kDenseMax / 2) + kDenseThreads - 1) / kDenseThreads;

// first pair index of row i of the k-vertex table
__device__ __forceinline__ int32_t dense_row_start(int32_t i, int32_t k) { return i * k - i * (i + 1) / 2; }

// Finishes the solve on the k = n_r <= kDenseMax components of round r, one
// workgroup: vertex u of the small graph is component u, edge {u, v} the
// lightest original edge between them, key pbest[pair_index(u, v)] (none: no
// edge; the key's low half is the edge index, or from round 2 on the
// position of its record).  Boruvka again, on that graph, with everything in
// LDS, contracting the graph after every round:
//   * every vertex takes its lightest key (row minimum, lane groups of 4);
//   * it hooks onto the vertex at the far end, except the smaller of a mutual
//     pair (both hold the same key, added once); pointer jumping flattens;
//   * the roots get new ids 0..k'-1 in id order, and the table is rebuilt for
//     the k' new vertices: entry {A, B} = minimum over the old entries whose
//     ends went to A and B (read into registers first, then LDS atomicMin
//     into the smaller table, which overlaps the old one).
// The keys are distinct, so the selected edges are exactly the MST edges
// between the k components; their key low halves are collected and marked in
// in_mst[] once at the end.  Records round r as the last one: n_{r+1} = 0,
// live_r = the surviving edges counted by the scan, sel_r = the edges added.
// LDS: table [np] u64, row minimum [k] u64, added key low halves [k] u32,
// parent [k] u16, target / new id [k] u16 (dense_finish_lds(k) bytes).
__global__ void __launch_bounds__(kDenseThreads) k_dense_finish(int round, int launched,
                                                               const unsigned long long* __restrict__ pbest,
                                                               const uint32_t* __restrict__ seg_live, int32_t nseg,
                                                               const uint4* __restrict__ rec,
                                                               uint8_t* __restrict__ in_mst, unsigned long long* total,
                                                               DevState* st, HostRound* host) {
  extern __shared__ unsigned long long dsm[];
  __shared__ unsigned long long red_w[kDenseWaves];
  __shared__ int64_t red_n[kDenseWaves];
  __shared__ int64_t red_l[kDenseWaves];
  __shared__ uint32_t nsel;
  __shared__ int32_t knext;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  // reads that depend on nothing else first: the scan's live counts and
  // the state tid 0 updates at the end
  int64_t live = 0;
  for (int32_t i0 = 0; i0 < nseg; i0 += 8 * kDenseThreads) {
    uint32_t v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int32_t i = i0 + q * kDenseThreads + tid;
      const uint32_t x = seg_live[i < nseg ? i : 0];  // nseg >= 1
      v[q] = i < nseg ? x : 0u;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) live += v[q];
  }
  int64_t added0 = 0;
  unsigned long long total0 = 0;
  if (tid == 0) {
    added0 = st->edges_added;
    total0 = *total;
  }
  const int32_t k0 = st->n[round];
  if (k0 <= 1 && round > 0) return;
  if (round > 0 && st->err) return;
  if (pick_mode(k0, launched) != kModeDense) return;
  const int32_t np0 = dense_pairs(k0);
  unsigned long long* tab = dsm;                                // [np0]
  unsigned long long* gbest = tab + np0;                        // [k0] row minimum
  uint32_t* selpos = reinterpret_cast<uint32_t*>(gbest + k0);   // [k0] low halves of the added keys
  uint16_t* par = reinterpret_cast<uint16_t*>(selpos + k0);     // [k0]
  uint16_t* tgt = par + k0;                                     // [k0] far end of the row minimum, then new id
  {
    // pbest holds kDensePairsMax keys (256-byte aligned): the clamped loads stay inside
    const ulonglong2* p2 = reinterpret_cast<const ulonglong2*>(pbest);
    const int32_t nq = np0 >> 1;
    ulonglong2 v[kDenseLoadIters];
#pragma unroll
    for (int q = 0; q < kDenseLoadIters; ++q) {
      const int32_t i = q * kDenseThreads + tid;
      v[q] = p2[i < nq ? i : 0];
    }
#pragma unroll
    for (int q = 0; q < kDenseLoadIters; ++q) {
      const int32_t i = q * kDenseThreads + tid;
      if (i < nq) {
        tab[2 * i] = v[q].x;
        tab[2 * i + 1] = v[q].y;
      }
    }
    if ((np0 & 1) && tid == 0) tab[np0 - 1] = pbest[np0 - 1];
  }
  if (tid == 0) nsel = 0;
  unsigned long long wsum = 0;
  int64_t added = 0;
  const int32_t u = tid / kDenseRowThreads;
  const int sub = tid % kDenseRowThreads;
  int32_t k = k0;
  __syncthreads();
  for (;;) {
    // row u: entries {v, u} for v < u at row_start(v) + u - v - 1 (the
    // start advances by 4k - 4v - 10 from v to v + 4), {u, v} for v > u at
    // row_start(u) + v - u - 1; lane `sub` takes v = sub, sub + 4, ...
    unsigned long long best = kKeyNone;
    int32_t arg = 0;
    if (u < k) {
      int32_t v = sub;
      int32_t rs = dense_row_start(sub, k);
#pragma unroll 4
      for (; v < u; v += kDenseRowThreads) {
        const unsigned long long key = tab[rs + u - v - 1];
        if (key < best) {
          best = key;
          arg = v;
        }
        rs += kDenseRowThreads * (k - v) - 10;
      }
      if (v == u) v += kDenseRowThreads;
      const int32_t base = dense_row_start(u, k) - u - 1;
#pragma unroll 4
      for (; v < k; v += kDenseRowThreads) {
        const unsigned long long key = tab[base + v];
        if (key < best) {
          best = key;
          arg = v;
        }
      }
    }
#pragma unroll
    for (int off = 1; off < kDenseRowThreads; off <<= 1) {
      const unsigned long long ok = __shfl_xor(best, off, 64);
      const int32_t oa = __shfl_xor(arg, off, 64);
      if (ok < best) {
        best = ok;
        arg = oa;
      }
    }
    const bool head = sub == 0 && u < k;
    if (head) {
      gbest[u] = best;
      tgt[u] = (uint16_t)arg;
      par[u] = (uint16_t)u;
    }
    if (!__syncthreads_or(head && best != kKeyNone)) break;  // no edge is left
    // hook: vertex g onto tgt[g], except the smaller vertex of a mutual pair
    for (int32_t g = tid; g < k; g += kDenseThreads) {
      const unsigned long long key = gbest[g];
      if (key != kKeyNone) {
        const int32_t t = tgt[g];
        if (!(tgt[t] == g && g < t)) {
          par[g] = (uint16_t)t;
          selpos[atomicAdd(&nsel, 1u)] = (uint32_t)key;
          wsum += key >> 32;
          ++added;
        }
      }
    }
    __syncthreads();
    // pointer jumping until every parent is a root
    for (;;) {
      bool changed = false;
      for (int32_t v = tid; v < k; v += kDenseThreads) {
        const int32_t p = par[v], pp = par[p];
        if (pp != p) {
          par[v] = (uint16_t)pp;
          changed = true;
        }
      }
      if (!__syncthreads_or(changed)) break;
    }
    // new ids of the roots that have an edge, in id order (one wave; k <=
    // 256).  A root without one is a vertex with no edge at all: it is done
    // and leaves the table, so k' <= k / 2.
    if (wv == 0) {
      int32_t nroots = 0;
      for (int32_t c0 = 0; c0 < k; c0 += 64) {
        const int32_t v = c0 + lane;
        const bool root = v < k && par[v] == v && gbest[v] != kKeyNone;
        const uint64_t mask = __ballot(root);
        if (root) tgt[v] = (uint16_t)(nroots + __popcll(mask & lanemask_lt()));
        nroots += __popcll(mask);
      }
      if (lane == 0) knext = nroots;
    }
    __syncthreads();
    const int32_t kn = knext;
    if (kn <= 1) break;
    // contraction: entry {i, j} (an edge: neither end is done) goes to
    // {A, B}, the new ids of the roots of i and j, unless A = B.  The new
    // table takes the top of the old one, [top, np): those old entries are
    // read into registers first, the ones below top straight from LDS after.
    const int32_t np = dense_pairs(k), npn = dense_pairs(kn), top = np - npn;
    auto new_index = [&](int32_t idx) -> int32_t {
      // row i of entry idx: the root of the quadratic, corrected by one step
      const float t = (float)(2 * k - 1);
      int32_t i = (int32_t)floorf((t - sqrtf(t * t - 8.0f * (float)idx)) * 0.5f);
      i = i < 0 ? 0 : i;
      if (dense_row_start(i, k) > idx) --i;
      if (dense_row_start(i + 1, k) <= idx) ++i;
      const int32_t j = idx - dense_row_start(i, k) + i + 1;
      const int32_t A = tgt[par[i]], B = tgt[par[j]];
      return A == B ? -1 : pair_index(A < B ? A : B, A < B ? B : A, kn);
    };
    unsigned long long ck[kDenseTopQ];
    int32_t ci[kDenseTopQ];
#pragma unroll
    for (int q = 0; q < kDenseTopQ; ++q) {
      const int32_t idx = top + q * kDenseThreads + tid;
      ck[q] = kKeyNone;
      ci[q] = -1;
      if (idx < np) {
        const unsigned long long key = tab[idx];
        if (key != kKeyNone) {
          ci[q] = new_index(idx);
          ck[q] = key;
        }
      }
    }
    __syncthreads();  // the top of the old table is in registers
    unsigned long long* ntab = tab + top;
    for (int32_t i = tid; i < npn; i += kDenseThreads) ntab[i] = kKeyNone;
    __syncthreads();
    for (int32_t idx = tid; idx < top; idx += kDenseThreads) {
      const unsigned long long key = tab[idx];
      if (key != kKeyNone) {
        const int32_t ni = new_index(idx);
        if (ni >= 0) atomicMin(&ntab[ni], key);
      }
    }
#pragma unroll
    for (int q = 0; q < kDenseTopQ; ++q)
      if (ci[q] >= 0) atomicMin(&ntab[ci[q]], ck[q]);
    tab = ntab;
    k = kn;
    __syncthreads();
  }
  // from round 2 on the key holds the record's position (the dense scan moves
  // no record; narrow records keep their edge indices apart), before that
  // the edge index
  const uint32_t nadd = nsel;
  const bool narrow_in = round >= 2 && st->n[round - 1] <= kNarrowMax;
  for (uint32_t i = tid; i < nadd; i += kDenseThreads) {
    const uint32_t x = selpos[i];
    const uint32_t e = round < 2 ? x
                       : (narrow_in ? reinterpret_cast<const uint32_t*>(rec)[narrow_e_index(x)] : rec[x].w);
    in_mst[e] = 1;
  }
  for (int off = 32; off > 0; off >>= 1) {
    wsum += __shfl_xor(wsum, off, 64);
    added += __shfl_xor(added, off, 64);
    live += __shfl_xor(live, off, 64);
  }
  if (lane == 0) {
    red_w[wv] = wsum;
    red_n[wv] = added;
    red_l[wv] = live;
  }
  __syncthreads();
  if (tid == 0) {
    unsigned long long W = 0;
    int64_t A = 0, Lv = 0;
    for (int i = 0; i < kDenseWaves; ++i) {
      W += red_w[i];
      A += red_n[i];
      Lv += red_l[i];
    }
    *total = total0 + W;
    st->live[round] = Lv;
    st->sel[round] = A;
    st->edges_added = added0 + A;
    st->n[round + 1] = 0;
    st->lab_off[round + 1] = st->lab_off[round];
    st->dense_at = round;
    HostRound h{0, st->err, st->err_internal, 1, Lv, A, added0 + A, st->stream[round], st->map_n[round],
                st->keep[round], 0, 0};
    host[round] = h;
    __threadfence_system();
  }
}

// ------------------------------------------------------------ sparse finish

// The cycle property of the dense finish, for a late round whose live edges
// join few distinct pairs of components (a sparse graph, e.g. a grid, has a
// few neighbours per component): only the lightest edge of every pair can
// be in the tree, so when the pairs fit one workgroup's LDS, Boruvka on the
// graph of components and pair-minimum edges ends the solve in one launch.
//
// k_pair_collect runs after an LDS-mode scan of round r >= 1 with n_r <=
// kSparseMaxK: it reads the records that scan left (narrow, with this
// round's labels, or kept with older ones, then mapped as the scan mapped
// them), and for every live one lowers the key of its pair {lo, hi} in an
// open-addressing table (slot claimed by compare-and-swap of the pair id,
// key lowered by an atomic minimum).  The key is the one the scan built: the
// weight and the record's position in the stream.  A probe sequence longer
// than kSparseProbes sets the overflow word; the finish counts the pairs
// against sparse_pair_cap(n_r).
__device__ __forceinline__ uint32_t pair_hash(uint32_t pid) {
  return (pid * 2654435761u) >> (32 - kSparseHashBits);
}

// Lowers the key of pair `pid` in the table: the slot is claimed (or found)
// by one compare-and-swap per probe, the key lowered by an atomic minimum
// whose result is not waited for.  True when no slot was found within
// kSparseProbes probes (overflow).  The finish counts the pairs.
__device__ __forceinline__ bool pair_insert(const SparseTable& sp, uint32_t pid, unsigned long long key) {
  uint32_t slot = pair_hash(pid);
  for (int probe = 0; probe < kSparseProbes; ++probe) {
    const uint32_t cur = atomicCAS(sp.pid + slot, kPairEmpty, pid);
    if (cur == kPairEmpty || cur == pid) {
      atomicMin(sp.key + slot, key);
      return false;
    }
    slot = (slot + 1) & (uint32_t)(kSparseHash - 1);
  }
  return true;
}

// Each workgroup first merges its segment's pairs in an LDS table of
// kPairLds slots (a segment of a late round's stream holds few distinct
// pairs: its edges are neighbours in the input order), lists the occupied
// slots, and inserts every distinct pair once into the global table, one
// list entry per thread at a time; a record that finds no LDS slot goes to
// the global table directly.
static constexpr int kPairLds = 2048;
static constexpr int kPairLdsProbes = 16;

__global__ void __launch_bounds__(kBlock) k_pair_collect(int round, int launched, const uint4* __restrict__ rec,
                                                         const int32_t* __restrict__ labpool,
                                                         const uint32_t* __restrict__ seg_cnt, int32_t nseg,
                                                         SparseTable sp, const DevState* __restrict__ st) {
  __shared__ uint32_t lpid[kPairLds];
  __shared__ unsigned long long lkey[kPairLds];
  __shared__ uint16_t list[kPairLds];
  __shared__ uint32_t nlist;
  if (round < 1) return;
  const int32_t nr = st->n[round];
  // tried where half the previous round's count is within kSparseMaxK: the
  // bound every round loop had when it enqueued this round (so every loop
  // tries the same rounds)
  if (nr <= 1 || st->n[round - 1] / 2 > kSparseMaxK) return;
  if (st->err || st->dense_at >= 0) return;
  if (pick_mode(nr, launched) != kModeLds) return;
  const bool kept = st->keep[round] == kKeepRecords;
  const int32_t* map = labpool + st->map_off[round];
  const unsigned long long* nrec = reinterpret_cast<const unsigned long long*>(rec);
  bool over = false;
  for (int32_t s = blockIdx.x; s < nseg; s += gridDim.x) {
    for (int i = threadIdx.x; i < kPairLds; i += kBlock) {
      lpid[i] = kPairEmpty;
      lkey[i] = kKeyNone;
    }
    if (threadIdx.x == 0) nlist = 0;
    __syncthreads();
    const uint32_t cnt = seg_cnt[s];
    const uint32_t base = (uint32_t)s * (uint32_t)kSegCap;
    for (uint32_t j = threadIdx.x; j < cnt; j += kBlock) {
      const unsigned long long x = nrec[narrow_rec_index(base + j)];
      int32_t a = (int32_t)(x & 0xFFFFu), b = (int32_t)((x >> 16) & 0xFFFFu);
      if (kept) {
        a = map[a];
        b = map[b];
      }
      if (a == b || (a | b) < 0 || a >= nr || b >= nr) continue;  // internal, isolated (or never: out of range)
      const uint32_t lo = (uint32_t)(a < b ? a : b), hi = (uint32_t)(a < b ? b : a);
      const uint32_t pid = lo * (uint32_t)nr + hi;
      const unsigned long long key = (x & 0xFFFFFFFF00000000ull) | (unsigned long long)(base + j);
      uint32_t slot = (pid * 2654435761u) >> (32 - 11);
      bool placed = false;
      for (int probe = 0; probe < kPairLdsProbes; ++probe) {
        uint32_t cur = atomicCAS(lpid + slot, kPairEmpty, pid);
        if (cur == kPairEmpty) list[atomicAdd(&nlist, 1u)] = (uint16_t)slot;
        if (cur == kPairEmpty || cur == pid) {
          lower_lds(lkey, (int32_t)slot, key);
          placed = true;
          break;
        }
        slot = (slot + 1) & (uint32_t)(kPairLds - 1);
      }
      if (!placed) over = pair_insert(sp, pid, key) || over;
    }
    __syncthreads();
    const uint32_t nl = nlist;
    for (uint32_t i = threadIdx.x; i < nl; i += kBlock) {
      const uint32_t slot = list[i];
      over = pair_insert(sp, lpid[slot], lkey[slot]) || over;
    }
    __syncthreads();  // the LDS table is reset for the next segment
  }
  if (over) atomicOr(sp.state + 1, 1u);
}
static_assert(kPairLds == 1 << 11, "LDS pair hash of 11 bits");

// One workgroup after k_pair_collect: if the pairs fit (no overflow), they
// are copied into LDS as a small graph -- the ends of every pair (2 + 2 B)
// and its key (8 B), per component its current root (2 B), lightest key
// (8 B), far end (2 B), parent (2 B) and the position of the key it added
// (4 B) -- and Boruvka runs to the end there: every root takes the lightest
// key over its pairs (LDS atomic minimum), the pair holding it names the far
// end (the keys are distinct), every root with an edge takes the far end's
// root as parent except the smaller of a mutual pair, pointer jumping
// flattens, every component reads its new root.  The added keys' positions
// give the edges (the narrow record at that position holds the edge index),
// marked in in_mst at the end; the round's record says the solve ended here
// (dense = 2).  Either way the table is emptied for a later round.
static constexpr int kSparseThreads = 1024;
static constexpr int kSparseJumpPasses = 40;

__global__ void __launch_bounds__(kSparseThreads) k_sparse_finish(int round, int launched,
                                                                 const uint4* __restrict__ rec, SparseTable sp,
                                                                 const uint32_t* __restrict__ seg_live, int32_t nseg,
                                                                 uint8_t* __restrict__ in_mst,
                                                                 unsigned long long* total, DevState* st,
                                                                 HostRound* host) {
  extern __shared__ unsigned long long fsm[];
  __shared__ uint32_t nsel_s;
  __shared__ uint32_t scan_sh[kScanWaves];
  __shared__ unsigned long long red_w[kSparseThreads / 64];
  __shared__ int64_t red_n[kSparseThreads / 64];
  __shared__ int64_t red_l[kSparseThreads / 64];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  int64_t live = 0;
  for (int32_t i0 = 0; i0 < nseg; i0 += 8 * kSparseThreads) {
    uint32_t v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int32_t i = i0 + q * kSparseThreads + tid;
      const uint32_t x = seg_live[i < nseg ? i : 0];  // nseg >= 1
      v[q] = i < nseg ? x : 0u;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) live += v[q];
  }
  int64_t added0 = 0;
  unsigned long long total0 = 0;
  if (tid == 0) {
    added0 = st->edges_added;
    total0 = *total;
  }
  if (round < 1) return;
  const int32_t k = st->n[round];
  // the same conditions as k_pair_collect: the table was filled iff they hold
  if (k <= 1 || st->n[round - 1] / 2 > kSparseMaxK) return;
  if (st->err || st->dense_at >= 0) return;
  if (pick_mode(k, launched) != kModeLds) return;
  const uint32_t cap = (uint32_t)sparse_pair_cap(k);
  const bool clean = sp.state[1] == 0;  // no probe sequence ran out
  // LDS: pair keys [cap] u64, component keys [k] u64, added positions [k]
  // u32, pair ends [cap] u16 x 2, root / far end / parent [k] u16 each
  unsigned long long* pkey = fsm;
  unsigned long long* ckey = pkey + cap;
  uint32_t* selpos = reinterpret_cast<uint32_t*>(ckey + k);
  uint16_t* pa = reinterpret_cast<uint16_t*>(selpos + k);
  uint16_t* pb = pa + cap;
  uint16_t* comp = pb + cap;
  uint16_t* far = comp + k;
  uint16_t* par = far + k;
  if (tid == 0) nsel_s = 0;
  // copy the occupied slots (as many as fit; all are counted) and empty the
  // table: this thread's 32 pair ids loaded first, then the keys of the
  // occupied ones; places in the pair list by a block-wide prefix sum of the
  // per-thread counts (one LDS counter for every pair would serialise)
  constexpr int kPer = kSparseHash / kSparseThreads;
  static_assert(kSparseHash % kSparseThreads == 0 && kPer == 32, "32 slots per thread");
  // every pair id of this thread's 32 slots loaded at once; the occupied
  // slots' indices go to the pair list's places (a block-wide prefix sum of
  // the per-thread counts, kept in pa[] for now), then the list is read
  // back, four entries per thread at a time, and each entry's pair id and
  // key loaded again (cache hits) into the list.  The occupied slots are
  // remembered (one bit each) and emptied at the very end: a barrier waits
  // for a workgroup's outstanding stores.
  uint32_t occupied = 0;
  {
    uint32_t pid[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) pid[q] = sp.pid[q * kSparseThreads + tid];
#pragma unroll
    for (int q = 0; q < kPer; ++q) occupied |= (pid[q] != kPairEmpty ? 1u : 0u) << q;
  }
  uint32_t base = 0;
  uint32_t at = block_excl_scan((uint32_t)__popc(occupied), scan_sh, &base);
  if (clean && base <= cap) {
#pragma unroll
    for (int q = 0; q < kPer; ++q)
      if ((occupied >> q) & 1u) pa[at++] = (uint16_t)(q * kSparseThreads + tid);
  }
  __syncthreads();
  if (clean && base <= cap) {
    for (uint32_t i0 = 0; i0 < base; i0 += 4 * kSparseThreads) {
      uint32_t slot[4], pid[4];
      unsigned long long key[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const uint32_t i = i0 + q * kSparseThreads + tid;
        slot[q] = i < base ? pa[i] : 0u;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        pid[q] = sp.pid[slot[q]];
        key[q] = sp.key[slot[q]];
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const uint32_t i = i0 + q * kSparseThreads + tid;
        if (i < base) {
          pkey[i] = key[q];
          pa[i] = (uint16_t)(pid[q] / (uint32_t)k);
          pb[i] = (uint16_t)(pid[q] % (uint32_t)k);
        }
      }
    }
  }
  const uint32_t npairs = base;
  const bool fits = clean && npairs <= cap;
  auto empty_table = [&]() {
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      if ((occupied >> q) & 1u) {
        sp.pid[q * kSparseThreads + tid] = kPairEmpty;
        sp.key[q * kSparseThreads + tid] = kKeyNone;
      }
    }
    if (tid < 2) sp.state[tid] = 0;
  };
  if (!fits) {
    empty_table();
    return;  // the round goes on with its one-workgroup close
  }
  for (int32_t v = tid; v < k; v += kSparseThreads) {
    comp[v] = (uint16_t)v;
    ckey[v] = kKeyNone;
  }
  __syncthreads();
  const uint32_t np = npairs;
  unsigned long long wsum = 0;
  int64_t added = 0;
  bool bad = false, finished = false;
  for (int it = 0; it < 64; ++it) {  // each pass at least halves the roots with an edge: ends far sooner
    // (the component keys are "none" here: set before the loop and at the
    // end of every pass)
    // four pairs per thread at a time, their loads issued together
    for (uint32_t i0 = 0; i0 < np; i0 += 4 * kSparseThreads) {
      int32_t a[4], b[4];
      unsigned long long key[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const uint32_t i = i0 + q * kSparseThreads + tid;
        const uint32_t ic = i < np ? i : 0u;
        a[q] = comp[pa[ic]];
        b[q] = comp[pb[ic]];
        key[q] = i < np ? pkey[ic] : kKeyNone;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (key[q] != kKeyNone && a[q] != b[q]) {
          lower_lds(ckey, a[q], key[q]);
          lower_lds(ckey, b[q], key[q]);
        }
      }
    }
    __syncthreads();
    for (uint32_t i0 = 0; i0 < np; i0 += 4 * kSparseThreads) {
      int32_t a[4], b[4];
      unsigned long long key[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const uint32_t i = i0 + q * kSparseThreads + tid;
        const uint32_t ic = i < np ? i : 0u;
        a[q] = comp[pa[ic]];
        b[q] = comp[pb[ic]];
        key[q] = i < np ? pkey[ic] : kKeyNone;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (key[q] != kKeyNone && a[q] != b[q]) {
          if (ckey[a[q]] == key[q]) far[a[q]] = (uint16_t)b[q];
          if (ckey[b[q]] == key[q]) far[b[q]] = (uint16_t)a[q];
        }
      }
    }
    __syncthreads();
    // hook; the added keys' places by one LDS atomic per wave
    bool any = false;
    for (int32_t c0 = 0; c0 < k; c0 += kSparseThreads) {
      const int32_t c = c0 + tid;
      bool hooks = false;
      unsigned long long key = kKeyNone;
      int32_t d = 0;
      if (c < k && comp[c] == c) {  // roots only
        key = ckey[c];
        par[c] = (uint16_t)c;
        if (key != kKeyNone) {
          d = far[c];
          hooks = !(far[d] == c && ckey[d] == key && c < d);  // the smaller of a mutual pair stays
        }
      }
      const uint64_t mask = __ballot(hooks);
      uint32_t base = 0;
      if (lane == 0 && mask) base = atomicAdd(&nsel_s, (uint32_t)__popcll(mask));
      base = __shfl(base, 0, 64);
      if (hooks) {
        par[c] = (uint16_t)d;
        selpos[base + (uint32_t)__popcll(mask & lanemask_lt())] = (uint32_t)key;
        wsum += key >> 32;
        ++added;
        any = true;
      }
    }
    if (!__syncthreads_or(any)) {
      finished = true;
      break;
    }
    bool jumping = true;
    int passes = 0;
    while (jumping && passes < kSparseJumpPasses) {
      bool changed = false;
      for (int32_t c = tid; c < k; c += kSparseThreads) {
        if (comp[c] != c) continue;
        const int32_t p = par[c], pp = par[p];
        if (pp != p) {
          par[c] = (uint16_t)pp;
          changed = true;
        }
      }
      jumping = __syncthreads_or(changed);
      ++passes;
    }
    bad = bad || jumping;  // still moving: a cycle, never expected
    for (int32_t v = tid; v < k; v += kSparseThreads) {
      comp[v] = par[comp[v]];
      ckey[v] = kKeyNone;  // for the next pass (read only by the hook, done)
    }
    __syncthreads();
  }
  bad = bad || !finished;
  const bool any_bad = __syncthreads_or(bad);
  for (int off = 32; off > 0; off >>= 1) {
    wsum += __shfl_xor(wsum, off, 64);
    added += __shfl_xor(added, off, 64);
    live += __shfl_xor(live, off, 64);
  }
  if (lane == 0) {
    red_w[wv] = wsum;
    red_n[wv] = added;
    red_l[wv] = live;
  }
  __syncthreads();
  if (tid == 0) {
    unsigned long long W = 0;
    int64_t A = 0, Lv = 0;
    for (int i = 0; i < kSparseThreads / 64; ++i) {
      W += red_w[i];
      A += red_n[i];
      Lv += red_l[i];
    }
    if (any_bad) st->err_internal = 1;
    *total = total0 + W;
    st->live[round] = Lv;
    st->sel[round] = A;
    st->edges_added = added0 + A;
    st->n[round + 1] = 0;
    st->lab_off[round + 1] = st->lab_off[round];
    st->dense_at = round;
    HostRound h{0, st->err, st->err_internal, 2, Lv, A, added0 + A, st->stream[round], st->map_n[round],
                st->keep[round], 0, 0};
    host[round] = h;
    __threadfence_system();
  }
  // after the last barrier: the edges of the added keys (the narrow record at
  // the position holds its index) and the emptied table
  const uint32_t nadd = nsel_s;
  const uint32_t* ne = reinterpret_cast<const uint32_t*>(rec);
  for (uint32_t i = tid; i < nadd; i += kSparseThreads) in_mst[ne[narrow_e_index(selpos[i])]] = 1;
  empty_table();
}

// -------------------------------------------------------------------- hook

// Root of x by plain loads (values may be stale, but every value ever stored
// in parent[] is an ancestor, so the walk ends at a node that was a root;
// a caller that links it checks that it still is).  Path halving with plain
// stores: only non-roots are written, always with an ancestor.
__device__ __forceinline__ int32_t walk_root(int32_t* parent, int32_t x) {
  int32_t p = parent[x];
  while (p != x) {
    const int32_t gp = parent[p];
    if (gp == p) return p;
    parent[x] = gp;
    x = gp;
    p = parent[x];
  }
  return x;
}

// For each component c with a minimum key: the edge e and d = the other
// end's component.  Round 0: the key holds e, and d = c ^ (src ^ dst of e),
// which the round-0 scan stored in the record buffer.  Later rounds: the key
// holds the edge's position in the record stream, whose record has this
// round's labels of both ends and e (a round that kept its narrow records
// in place finds the labels of the round that wrote them there, and maps
// them through its label map).
// Hooking by successors: c's parent becomes d.  Following the lightest
// edges from any component reaches exactly one pair of components that chose
// each other (the keys are distinct and strictly decrease along the way), so
// the only cycles are those mutual pairs; the smaller component of a pair
// stays a root.  The parents then form a forest whose trees are the merged
// components, with plain stores only (each thread writes its own entry).
// Every component that got a parent owns its edge: a mutual pair's common
// edge is marked once (by the larger), every other selected edge by the one
// component that chose it.  k_compress finds the roots.
__global__ void __launch_bounds__(kBlock) k_hook(int round, const uint4* __restrict__ rec,
                                                 const int32_t* __restrict__ labpool,
                                                 const unsigned long long* __restrict__ best,
                                                 int32_t* __restrict__ parent, DevState* __restrict__ st,
                                                 uint8_t* __restrict__ in_mst, uint32_t* __restrict__ part_sel,
                                                 unsigned long long* __restrict__ part_w) {
  __shared__ uint32_t red32[kBlock / 64];
  __shared__ unsigned long long red64[kBlock / 64];
  const int32_t nr = st->n[round];
  if (nr <= 1 && round > 0) return;
  if (st->dense_at == round) return;  // the dense finish ended the solve
  const bool narrow = nr <= kNarrowMax;        // the records at the keys' positions are narrow
  const bool keep = st->keep[round] == kKeepRecords;  // ... and hold the labels of the round that wrote them
  const int32_t* map = labpool + st->map_off[round];
  uint32_t sel = 0;
  unsigned long long wsum = 0;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t ci = (int64_t)blockIdx.x * kBlock + threadIdx.x; ci < nr; ci += stride) {
    const int32_t c = (int32_t)ci;
    const unsigned long long key = best[c];
    if (key == kKeyNone) continue;
    int32_t u, v;
    uint32_t e;
    int32_t d;
    if (round == 0) {
      // the round-0 scan stored src ^ dst of every edge in the record buffer
      e = (uint32_t)key;
      d = (int32_t)(reinterpret_cast<const uint32_t*>(rec)[e] ^ (uint32_t)c);
      u = c;
      v = d;
    } else {
      const uint32_t pos = (uint32_t)key;
      if (narrow) {
        const unsigned long long x = reinterpret_cast<const unsigned long long*>(rec)[narrow_rec_index(pos)];
        e = reinterpret_cast<const uint32_t*>(rec)[narrow_e_index(pos)];
        u = (int32_t)(x & 0xFFFFu);
        v = (int32_t)((x >> 16) & 0xFFFFu);
        if (keep) {
          u = map[u];
          v = map[v];
        }
      } else {
        const uint4 x = ld_rec(rec + pos);
        u = (int32_t)x.x;
        v = (int32_t)x.y;
        e = x.w;
      }
      d = (u == c) ? v : u;
    }
    if ((uint32_t)d >= (uint32_t)nr || d == c || (u != c && v != c)) {
      st->err_internal = 1;  // inconsistent labels: never expected, reported as a device error
      continue;
    }
    // d > c: c stays a root if d chose the same edge (a mutual pair)
    if (d > c && best[d] == key) continue;
    parent[c] = d;
    in_mst[e] = 1;
    ++sel;
    wsum += (uint32_t)(key >> 32);  // the edge's weight
  }
  sel = block_sum<kBlock / 64>(sel, red32);
  wsum = block_sum<kBlock / 64>(wsum, red64);
  if (threadIdx.x == 0) {
    part_sel[blockIdx.x] = sel;
    part_w[blockIdx.x] = wsum;
  }
}

// ---------------------------------------------------------------- compress

// root_of[c] = root of c (path halving with plain accesses; every value
// written is an ancestor).  One wave handles 64 consecutive components; its
// ballot of "root with an outgoing edge" is rootmask[c / 64], its popcount
// rootcnt[c / 64].  A root without a minimum edge is an isolated component:
// it is final and gets no new label.
__global__ void __launch_bounds__(kBlock) k_compress(int round, int32_t* parent,
                                                     int32_t* __restrict__ root_of,
                                                     const unsigned long long* __restrict__ best,
                                                     unsigned long long* __restrict__ rootmask,
                                                     int32_t* __restrict__ rootcnt,
                                                     const DevState* __restrict__ st) {
  const int32_t nr = st->n[round];
  if (nr <= 1 && round > 0) return;
  if (st->dense_at == round) return;  // the dense finish ended the solve
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t base = (int64_t)blockIdx.x * kBlock + (threadIdx.x & ~63); base < nr; base += stride) {
    const int64_t ci = base + lane_id();
    bool keep = false;
    if (ci < nr) {
      const int32_t c = (int32_t)ci;
      const int32_t root = walk_root(parent, c);
      root_of[c] = root;
      keep = (root == c) && (best[c] != kKeyNone);
    }
    const uint64_t mask = __ballot(keep);
    if (lane_id() == 0) {
      rootmask[base >> 6] = mask;
      rootcnt[base >> 6] = (int32_t)__popcll(mask);
    }
  }
}

// ---------------------------------------------------------------- finalize

// The stream state round r leaves for round r + 1 (one thread; n_next
// components enter round r + 1; `in` is the state as round r found it,
// written to st): the records it reads (`stream_next`), the
// map from the labels in the records to round r + 1's (round r's own label
// map if round r rewrote the records, else that map composed with round r's,
// which k_relabel / k_round_tail write), and what round r + 1 does with its
// records: narrow records, fewer than 1/kKeepDeadDen of the records round r
// read dead there, are kept in place if every LDS or dense launch of round
// r + 2 (bound n_next / 2) can stage the composed map it would then read,
// else relabelled in place; otherwise the survivors are compacted.
__device__ __forceinline__ int next_stream_state(const DevState& in, DevState* st, int round, int32_t nr,
                                                 int32_t n_next, int64_t live, int64_t stream_next) {
  const int64_t read = in.stream[round];
  const bool kept = in.keep[round] == kKeepRecords;
  const int64_t map_off = kept ? in.cmap_off + (int64_t)((round + 1) & 1) * kNarrowMax : in.lab_off[round];
  const int32_t map_n = kept ? in.map_n[round] : nr;
  int what = kMoveRecords;
  if (round >= 1 && nr <= kNarrowMax && (int64_t)kKeepDeadDen * (read - live) < read) {
    const int64_t bound = n_next / 2;
    const int modes = scan_modes(bound, false, 3, in.dense_limit, true, kBucketMaxComponents);
    bool fits = true;
    for (int mode : {kModeLds, kModeDense})
      if ((modes >> mode) & 1) fits = fits && map_fits_lds(mode, bound, in.dense_limit, map_n);
    what = fits ? kKeepRecords : kRelabelRecords;
  }
  st->stream[round + 1] = stream_next;
  st->map_off[round + 1] = map_off;
  st->map_n[round + 1] = map_n;
  st->keep[round + 1] = what;
  return what;
}

// Stores the 16 prefixes of words g0 .. g0 + 15 (those below W).
__device__ __forceinline__ void store_prefixes(int32_t* rootpre, int32_t g0, int32_t W, const int32_t (&pre)[16]) {
  if (g0 + 15 < W) {
#pragma unroll
    for (int k = 0; k < 4; ++k)
      *reinterpret_cast<int4*>(rootpre + g0 + 4 * k) = make_int4(pre[4 * k], pre[4 * k + 1], pre[4 * k + 2],
                                                                   pre[4 * k + 3]);
  } else {
#pragma unroll
    for (int k = 0; k < 16; ++k)
      if (g0 + k < W) rootpre[g0 + k] = pre[k];
  }
}

// One workgroup of 1024 threads.  Exclusive scan of rootcnt[0..W) into
// rootpre, W = ceil(n_r / 64); n_{r+1} = total.  Reduces this round's
// per-segment counts: live edges (seg_live) and records in the stream
// (seg_cnt), and the per-block partials of the hook: edges added and their
// weight (part_sel / part_w [0..nhook)); adds the weight to *total; writes
// the round's record for the host (pinned host memory) and the stream state
// of the next round.  The kernel is a chain of dependent memory round trips,
// so every independent read is issued at entry: the device state (copied to
// LDS, one word per thread), the running total, the counts and partials
// (several per thread in flight); the root counts follow once n_r is known,
// 16 consecutive words per thread (four 16-byte loads) per pass.  A barrier
// waits for the workgroup's outstanding stores, so the stores come after the
// last one (the prefixes of the last pass stay in registers until then).
__global__ void __launch_bounds__(1024) k_finalize(int round, const int32_t* __restrict__ rootcnt,
                                                   int32_t* __restrict__ rootpre,
                                                   const uint32_t* __restrict__ seg_cnt,
                                                   const uint32_t* __restrict__ seg_live, int32_t nseg,
                                                   const uint32_t* __restrict__ part_sel,
                                                   const unsigned long long* __restrict__ part_w,
                                                   int32_t nhook, DevState* st,
                                                   unsigned long long* total, HostRound* host) {
  __shared__ DevState sst;  // the device state as this kernel found it
  __shared__ int64_t sh[16];
  __shared__ int64_t sh_live[16], sh_recs[16], sh_sel[16];
  __shared__ unsigned long long sh_w[16];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  {
    constexpr int kWords = (int)(sizeof(DevState) / 4);
    static_assert(sizeof(DevState) % 4 == 0 && kWords <= 1024, "one word of the state per thread");
    if (tid < kWords) reinterpret_cast<uint32_t*>(&sst)[tid] = reinterpret_cast<const uint32_t*>(st)[tid];
  }
  const unsigned long long total0 = tid == 0 ? *total : 0ull;
  // counts and partials (nseg >= 1 and nhook >= 1: clamped reads stay inside)
  int64_t live = 0, recs = 0, sel = 0;
  unsigned long long ws = 0;
  for (int32_t i0 = 0; i0 < nseg; i0 += 8 * 1024) {
    uint32_t v[8], c[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int32_t i = i0 + q * 1024 + tid;
      const uint32_t x = seg_live[i < nseg ? i : 0];
      const uint32_t y = seg_cnt[i < nseg ? i : 0];
      v[q] = i < nseg ? x : 0u;
      c[q] = i < nseg ? y : 0u;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      live += v[q];
      recs += c[q];
    }
  }
  for (int32_t i0 = 0; i0 < nhook; i0 += 4 * 1024) {
    uint32_t c[4];
    unsigned long long x[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int32_t i = i0 + q * 1024 + tid;
      const int32_t ic = i < nhook ? i : 0;
      c[q] = part_sel[ic];
      x[q] = part_w[ic];
      if (i >= nhook) {
        c[q] = 0;
        x[q] = 0;
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      sel += c[q];
      ws += x[q];
    }
  }
  live = wave_sum(live);
  recs = wave_sum(recs);
  sel = wave_sum(sel);
  ws = wave_sum(ws);
  if (lane == 0) {
    sh_live[wv] = live;
    sh_recs[wv] = recs;
    sh_sel[wv] = sel;
    sh_w[wv] = ws;
  }
  __syncthreads();  // the state's copy and the per-wave sums are complete
  const int32_t nr = sst.n[round];
  if (sst.dense_at == round) return;  // the dense finish wrote this round's record
  if (nr <= 1 && round > 0) {
    if (tid == 0) {
      st->n[round + 1] = 0;
      st->lab_off[round + 1] = sst.lab_off[round];
      HostRound h{0, sst.err, sst.err_internal, 0, 0, 0, sst.edges_added, 0, 0, 0, 0, 0};
      host[round] = h;
      __threadfence_system();
    }
    return;
  }
  // passes of 1024 x 16 words: exclusive scan with a carry
  const int32_t W = (nr + 63) >> 6;
  int64_t carry = 0;
  int32_t pre[16];
  int32_t g_last = W;  // first word of this thread's prefixes still to store (W: none)
  for (int32_t t0 = 0; t0 < W; t0 += 16 * 1024) {
    const int32_t g0 = t0 + 16 * tid;
    int32_t v[16];
    if (g0 + 15 < W) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int4 q = *reinterpret_cast<const int4*>(rootcnt + g0 + 4 * k);
        v[4 * k] = q.x;
        v[4 * k + 1] = q.y;
        v[4 * k + 2] = q.z;
        v[4 * k + 3] = q.w;
      }
    } else {
#pragma unroll
      for (int k = 0; k < 16; ++k) v[k] = g0 + k < W ? rootcnt[g0 + k] : 0;
    }
    int64_t mine = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) mine += v[k];
    int64_t x = mine;
    for (int off = 1; off < 64; off <<= 1) {
      const int64_t y = __shfl_up(x, off, 64);
      if (lane >= off) x += y;
    }
    if (lane == 63) sh[wv] = x;
    __syncthreads();
    int64_t wave_base = 0, tile_tot = 0;
    for (int i = 0; i < 16; ++i) {
      wave_base += (i < wv) ? sh[i] : 0;
      tile_tot += sh[i];
    }
    int64_t e = carry + wave_base + x - mine;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      pre[k] = (int32_t)e;
      e += v[k];
    }
    carry += tile_tot;
    g_last = g0;
    if (t0 + 16 * 1024 < W) {
      // another pass follows: store now (sh[] is rewritten by that pass)
      store_prefixes(rootpre, g0, W, pre);
      g_last = W;
      __syncthreads();
    }
  }
  if (tid == 0) {
    int64_t L = 0, Rn = 0, T = 0;
    unsigned long long S = 0;
    for (int i = 0; i < 16; ++i) {
      L += sh_live[i];
      Rn += sh_recs[i];
      T += sh_sel[i];
      S += sh_w[i];
    }
    const int64_t total_roots = carry;
    const int64_t added = sst.edges_added + T;
    st->live[round] = L;
    st->sel[round] = T;
    st->edges_added = added;
    st->n[round + 1] = (int32_t)total_roots;
    st->lab_off[round + 1] = sst.lab_off[round] + nr;
    *total = total0 + S;
    // round 0 leaves the stream untouched: round 1 reads the caller's edges
    const int next = next_stream_state(sst, st, round, nr, (int32_t)total_roots, L, round == 0 ? sst.m : Rn);
    HostRound h{(int32_t)total_roots, sst.err, sst.err_internal, 0,
                L,                    T,       added,            sst.stream[round],
                sst.map_n[round],     sst.keep[round], next,     0};
    host[round] = h;
    __threadfence_system();
  }
  if (g_last < W) store_prefixes(rootpre, g_last, W, pre);
}

// ----------------------------------------------------------------- relabel

// lab_r[c] = dense new label of c's root: the number of kept roots with a
// smaller id (rootpre of its 64-word plus a popcount inside the word); -1 for
// an isolated component.  When round r kept its records, the map round r + 1
// applies to them is lab_r composed with round r's map (the same label of
// the root, reached through that map).  Then parent[] and best[] are reset
// for the n_{r+1} components of the next round.
__global__ void __launch_bounds__(kBlock) k_relabel(int round, const int32_t* __restrict__ root_of,
                                                    const unsigned long long* __restrict__ rootmask,
                                                    const int32_t* __restrict__ rootpre,
                                                    int32_t* __restrict__ labpool, int32_t* parent,
                                                    unsigned long long* best, uint32_t* __restrict__ btot,
                                                    const DevState* __restrict__ st) {
  const int32_t nr = st->n[round];
  if (nr <= 1 && round > 0) return;
  if (st->dense_at == round) return;  // the dense finish ended the solve
  const int32_t nn = st->n[round + 1];
  const int64_t off = st->lab_off[round];
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  auto label_of = [&](int32_t c) -> int32_t {
    const int32_t r = root_of[c];
    const unsigned long long word = rootmask[r >> 6];
    const int bit = r & 63;
    return ((word >> bit) & 1ull) ? rootpre[r >> 6] + __popcll(word & ((1ull << bit) - 1ull)) : -1;
  };
  for (int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x; c < nr; c += stride)
    labpool[off + c] = label_of((int32_t)c);
  if (st->keep[round] == kKeepRecords) {
    const int32_t* mi = labpool + st->map_off[round];
    int32_t* mo = labpool + st->map_off[round + 1];
    const int32_t ne = st->map_n[round];
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < ne; i += stride) {
      const int32_t x = mi[i];
      mo[i] = x < 0 ? -1 : label_of(x);
    }
  }
  for (int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x; c < nn; c += stride) {
    parent[c] = (int32_t)c;
    best[c] = kKeyNone;
  }
  if (btot)
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < kMaxBuckets; i += stride) btot[i] = 0;
}

// -------------------------------------------------------- small round tail

// Hook, compress, finalize and relabel of one round in one workgroup, for a
// round with n_r <= kTailMax components (the host launches it only when its
// bound on n_r is that small).  The same steps as k_hook .. k_relabel, with
// the parent forest in LDS: every component with a minimum edge takes the
// component at the far end as its parent, except the smaller of a mutual
// pair, which stays a root (the rule of k_hook, so the roots and labels --
// rank among the kept roots, -1 for an isolated component -- equal the
// multi-kernel path's).  The roots are then found by pointer jumping: every
// pass replaces each parent by its parent's parent, so a chain of length L
// is resolved in about log2 L passes (a walk along it would take L dependent
// LDS reads, and the minimum edges of grid-like graphs form long chains).
// LDS: parent [n_r] and target / root [n_r], int32 each.
static constexpr int kTailJumpPasses = 40;  // > log2(kTailMax) + 2: more means a cycle, an internal error
static constexpr int kTailThreads = 1024;
static constexpr int kTailPer = (kTailMax + kTailThreads - 1) / kTailThreads;

__global__ void __launch_bounds__(kTailThreads) k_round_tail(int round, int32_t cap, const uint4* __restrict__ rec,
                                                            unsigned long long* best, int32_t* parent,
                                                            int32_t* __restrict__ labpool,
                                                            const uint32_t* __restrict__ seg_cnt,
                                                            const uint32_t* __restrict__ seg_live, int32_t nseg,
                                                            uint8_t* __restrict__ in_mst,
                                                            unsigned long long* total, uint32_t* __restrict__ btot,
                                                            DevState* st, HostRound* host) {
  extern __shared__ int32_t tsm[];
  __shared__ int64_t red_a[kTailThreads / 64];
  __shared__ int64_t red_b[kTailThreads / 64];
  __shared__ int64_t red_c[kTailThreads / 64];
  __shared__ int64_t red_l[kTailThreads / 64];
  __shared__ unsigned long long red_w[kTailThreads / 64];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  // Every read that does not depend on another is issued here, before the
  // first use: the round's count and state, the minimum keys of components
  // below the host's bound cap (<= the vertex count, so inside best[]), the
  // scan's survivor counts.
  const int32_t nr = st->n[round];
  const int32_t dense_at = st->dense_at;
  unsigned long long key[kTailPer];
#pragma unroll
  for (int q = 0; q < kTailPer; ++q) {
    const int32_t c = tid + q * kTailThreads;
    const unsigned long long k = best[c < cap ? c : 0];
    key[q] = c < cap ? k : kKeyNone;
  }
  int64_t live = 0, recs = 0;
  for (int32_t i0 = 0; i0 < nseg; i0 += 8 * kTailThreads) {
    uint32_t v[8], c[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int32_t i = i0 + q * kTailThreads + tid;
      const uint32_t x = seg_live[i < nseg ? i : 0];  // nseg >= 1
      const uint32_t y = seg_cnt[i < nseg ? i : 0];
      v[q] = i < nseg ? x : 0u;
      c[q] = i < nseg ? y : 0u;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      live += v[q];
      recs += c[q];
    }
  }
  const int64_t off = st->lab_off[round];
  int64_t added0 = 0;
  unsigned long long total0 = 0;
  int err0 = 0, erri0 = 0;
  if (tid == 0) {
    added0 = st->edges_added;
    total0 = *total;
    err0 = st->err;
    erri0 = st->err_internal;
  }
  if (dense_at == round) return;  // the dense finish wrote this round's record
  if (nr <= 1 && round > 0) {
    if (tid == 0) {
      st->n[round + 1] = 0;
      st->lab_off[round + 1] = off;
      HostRound h{0, err0, erri0, 0, 0, 0, added0, 0, 0, 0, 0, 0};
      host[round] = h;
      __threadfence_system();
    }
    return;
  }
  if (nr > cap) {  // never: the host's bound covers n_r
    if (tid == 0) {
      st->err_internal = 1;
      HostRound h{0, err0, 1, 0, 0, 0, added0, 0, 0, 0, 0, 0};
      host[round] = h;
      __threadfence_system();
    }
    return;
  }
  int32_t* par = tsm;       // [nr]
  int32_t* tgt = tsm + nr;  // [nr] far end of the minimum edge (-1: none), then the root
#pragma unroll
  for (int q = 0; q < kTailPer; ++q)
    if (tid + q * kTailThreads >= nr) key[q] = kKeyNone;
  // the records of the minimum edges of components tid, tid + 1024, ...: all
  // loads issued (unconditionally, clamped to slot 0) before any is used
  int32_t d[kTailPer];
  uint32_t e[kTailPer];
  bool bad = false;
  if (round == 0) {
    // the round-0 scan stored src ^ dst of every edge in the record buffer
    const uint32_t* xends = reinterpret_cast<const uint32_t*>(rec);
    uint32_t xv[kTailPer];
#pragma unroll
    for (int q = 0; q < kTailPer; ++q) xv[q] = xends[key[q] != kKeyNone ? (uint32_t)key[q] : 0u];
#pragma unroll
    for (int q = 0; q < kTailPer; ++q) {
      const int32_t c = tid + q * kTailThreads;
      e[q] = (uint32_t)key[q];
      d[q] = key[q] != kKeyNone ? (int32_t)(xv[q] ^ (uint32_t)c) : -1;
    }
  } else {
    // the record at the key's position: wide, or narrow (this round's labels
    // when the scan rewrote it, else those of the round that wrote it,
    // mapped through this round's label map)
    uint2 ab[kTailPer];
    if (nr <= kNarrowMax) {
      const unsigned long long* nrec = reinterpret_cast<const unsigned long long*>(rec);
      const uint32_t* ne = reinterpret_cast<const uint32_t*>(rec);
#pragma unroll
      for (int q = 0; q < kTailPer; ++q) {
        const uint32_t pos = key[q] != kKeyNone ? (uint32_t)key[q] : 0u;
        const unsigned long long x = nrec[narrow_rec_index(pos)];
        e[q] = ne[narrow_e_index(pos)];
        ab[q] = make_uint2((uint32_t)(x & 0xFFFFu), (uint32_t)((x >> 16) & 0xFFFFu));
      }
      if (st->keep[round] == kKeepRecords) {
        const int32_t* map = labpool + st->map_off[round];
#pragma unroll
        for (int q = 0; q < kTailPer; ++q) ab[q] = make_uint2((uint32_t)map[ab[q].x], (uint32_t)map[ab[q].y]);
      }
    } else {
#pragma unroll
      for (int q = 0; q < kTailPer; ++q) {
        const uint32_t pos = key[q] != kKeyNone ? (uint32_t)key[q] : 0u;
        ab[q] = *reinterpret_cast<const uint2*>(rec + pos);
        e[q] = rec[pos].w;
      }
    }
#pragma unroll
    for (int q = 0; q < kTailPer; ++q) {
      const int32_t c = tid + q * kTailThreads;
      const int32_t u = (int32_t)ab[q].x, v = (int32_t)ab[q].y;
      d[q] = key[q] == kKeyNone ? -1 : (u == c ? v : u);
      if (key[q] != kKeyNone && u != c && v != c) {
        bad = true;  // inconsistent labels: never expected, reported as a device error
        d[q] = -1;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < kTailPer; ++q) {
    if (key[q] != kKeyNone && (uint32_t)d[q] >= (uint32_t)nr) {
      bad = true;
      d[q] = -1;
    }
  }
#pragma unroll
  for (int q = 0; q < kTailPer; ++q) {
    const int32_t c = tid + q * kTailThreads;
    if (c < nr) {
      par[c] = c;
      tgt[c] = d[q];
    }
  }
  const bool any_bad0 = __syncthreads_or(bad);
  // hook by successors; of a mutual pair (each the other's far end, so the
  // same edge) the larger id hooks and owns the edge.  Global stores wait
  // until after the last barrier (a barrier waits for them): the edges this
  // thread adds are remembered in a bit mask.
  uint32_t sel = 0, hooked = 0;
  unsigned long long wsum = 0;
#pragma unroll
  for (int q = 0; q < kTailPer; ++q) {
    const int32_t c = tid + q * kTailThreads;
    if (c >= nr) continue;
    const bool hooks = d[q] >= 0 && !(d[q] > c && tgt[d[q]] == c);
    par[c] = hooks ? d[q] : c;
    if (hooks) {
      hooked |= 1u << q;
      ++sel;
      wsum += (uint32_t)(key[q] >> 32);  // the edge's weight
    }
  }
  // the round's sums, per wave (read by thread 0 after the last barrier)
  live = wave_sum(live);
  recs = wave_sum(recs);
  const int64_t sel64 = wave_sum((int64_t)sel);
  wsum = wave_sum(wsum);
  if (lane == 0) {
    red_b[wv] = sel64;
    red_c[wv] = recs;
    red_l[wv] = live;
    red_w[wv] = wsum;
  }
  __syncthreads();
  // pointer jumping in place: a value read while another thread rewrites it
  // is the old or the new parent, both ancestors, so every pass keeps each
  // entry on its path to the root and the passes end when none changes
  bool jumping = true;
  int passes = 0;
  while (jumping && passes < kTailJumpPasses) {
    bool changed = false;
#pragma unroll
    for (int q = 0; q < kTailPer; ++q) {
      const int32_t c = tid + q * kTailThreads;
      if (c >= nr) continue;
      const int32_t p = __hip_atomic_load(par + c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      const int32_t pp = __hip_atomic_load(par + p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      if (pp != p) {
        __hip_atomic_store(par + c, pp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        changed = true;
      }
    }
    jumping = __syncthreads_or(changed);
    ++passes;
  }
  const bool any_bad = any_bad0 || jumping;  // still moving: a cycle, never expected
  // roots: tgt[c] = root of c, -1 for an isolated component (no minimum
  // edge: nothing hooked onto it and it hooked onto nothing)
#pragma unroll
  for (int q = 0; q < kTailPer; ++q) {
    const int32_t c = tid + q * kTailThreads;
    if (c < nr) tgt[c] = d[q] < 0 && par[c] == c ? -1 : par[c];
  }
  __syncthreads();
  // new labels: rank of each kept root (tgt[c] == c) in id order; thread t
  // ranks components t * kTailPer .. t * kTailPer + kTailPer - 1, into par[]
  int32_t mine = 0;
#pragma unroll
  for (int q = 0; q < kTailPer; ++q) {
    const int32_t c = tid * kTailPer + q;
    if (c < nr && tgt[c] == c) ++mine;
  }
  int32_t x = mine;
  for (int off = 1; off < 64; off <<= 1) {
    const int32_t y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) red_a[wv] = x;
  __syncthreads();
  int32_t rank = x - mine, roots = 0;
  for (int i = 0; i < kTailThreads / 64; ++i) {
    rank += i < wv ? (int32_t)red_a[i] : 0;
    roots += (int32_t)red_a[i];
  }
#pragma unroll
  for (int q = 0; q < kTailPer; ++q) {
    const int32_t c = tid * kTailPer + q;
    if (c < nr && tgt[c] == c) par[c] = rank++;
  }
  __syncthreads();  // the last barrier: global stores from here on
  if (tid == 0) {
    int64_t L = 0, T = 0, R = 0;
    unsigned long long W = 0;
    for (int i = 0; i < kTailThreads / 64; ++i) {
      L += red_l[i];
      T += red_b[i];
      R += red_c[i];
      W += red_w[i];
    }
    const int erri = any_bad ? 1 : erri0;
    st->err_internal = erri;
    st->live[round] = L;
    st->sel[round] = T;
    st->edges_added = added0 + T;
    st->n[round + 1] = roots;
    st->lab_off[round + 1] = off + nr;
    *total = total0 + W;
    const int next = next_stream_state(*st, st, round, nr, roots, L, round == 0 ? st->m : R);
    HostRound h{roots, err0, erri, 0, L, T, added0 + T, st->stream[round], st->map_n[round], st->keep[round],
                next, 0};
    host[round] = h;
    __threadfence_system();
  }
#pragma unroll
  for (int q = 0; q < kTailPer; ++q) {
    const int32_t c = tid + q * kTailThreads;
    if (c < nr) {
      const int32_t r = tgt[c];
      labpool[off + c] = r < 0 ? -1 : par[r];
      if ((hooked >> q) & 1u) in_mst[e[q]] = 1;
    }
  }
  if (st->keep[round] == kKeepRecords) {
    // the records stay as they are: the next round's map is this round's
    // map composed with the labels just given
    const int32_t* mi = labpool + st->map_off[round];
    int32_t* mo = labpool + st->cmap_off + (int64_t)((round + 1) & 1) * kNarrowMax;
    const int32_t ne = st->map_n[round];
    for (int32_t i0 = 0; i0 < ne; i0 += 8 * kTailThreads) {
      int32_t x[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int32_t i = i0 + q * kTailThreads + tid;
        x[q] = mi[i < ne ? i : 0];
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int32_t i = i0 + q * kTailThreads + tid;
        const int32_t r = x[q] < 0 ? -1 : tgt[x[q]];
        if (i < ne) mo[i] = r < 0 ? -1 : par[r];
      }
    }
  }
  // the next round's parent[] and best[] (n_{r+1} = roots), bucket counters
  for (int32_t c = tid; c < roots; c += kTailThreads) {
    parent[c] = c;
    best[c] = kKeyNone;
  }
  if (btot)
    for (int32_t i = tid; i < kMaxBuckets; i += kTailThreads) btot[i] = 0;
}

// ------------------------------------------------------------ launchers

#define MSTX_LAUNCH_CHECK()            \
  do {                                 \
    hipError_t _e = hipGetLastError(); \
    if (_e != hipSuccess) return _e;   \
  } while (0)

template <int M, int St>
static hipError_t raise_lds_limit() {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_scan<M, St>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxDynLds);
}

hipError_t configure_kernels() {
  hipError_t e = hipSuccess;
#define MSTX_CFG(M)                                                        \
  do {                                                                     \
    for (hipError_t r_ : {raise_lds_limit<M, 0>(), raise_lds_limit<M, 1>(), \
                          raise_lds_limit<M, 2>(), raise_lds_limit<M, 3>()}) \
      if (r_ != hipSuccess) e = r_;                                        \
  } while (0)
  MSTX_CFG(kModeLds);
  MSTX_CFG(kModeBucket);
  MSTX_CFG(kModeDense);
#undef MSTX_CFG
  hipError_t r4 = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_round_tail),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxDynLds);
  if (r4 != hipSuccess) e = r4;
  hipError_t r3 = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_dense_finish),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxDynLds);
  if (r3 != hipSuccess) e = r3;
  hipError_t r2 = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_bucket_min),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxDynLds);
  if (r2 != hipSuccess) e = r2;
  hipError_t r5 = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_sparse_finish),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxDynLds);
  if (r5 != hipSuccess) e = r5;
  return e;
}

hipError_t launch_init(int32_t n, int64_t m, int64_t cmap_off, int dense_limit, unsigned long long* best,
                       int32_t* parent, unsigned long long* pbest, uint32_t* btot, SparseTable sp, DevState* st,
                       int grid, hipStream_t s) {
  k_init<<<grid, kBlock, 0, s>>>(n, m, cmap_off, dense_limit, best, parent, pbest, btot, sp, st);
  MSTX_LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_fill_u8(uint8_t* p, int64_t count, uint8_t v, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const int64_t blocks = (count + 16 * kBlock - 1) / (16 * kBlock);
  k_fill_u8<<<(int)(blocks < 4096 ? blocks : 4096), kBlock, 0, s>>>(p, count, v);
  MSTX_LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_fill_u64(unsigned long long* p, int64_t count, unsigned long long v, int grid, hipStream_t s) {
  k_fill_u64<<<grid, kBlock, 0, s>>>(p, count, v);
  MSTX_LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_scan(int mode, int stage, const ScanArgs& a, int grid, size_t lds, hipStream_t s) {
  // stage: the edge stream the round reads (scan_stage)
#define MSTX_SCAN(M)                                                    \
  do {                                                                  \
    if (stage == 0) k_scan<M, 0><<<grid, kScanBlock, lds, s>>>(a);      \
    else if (stage == 1) k_scan<M, 1><<<grid, kScanBlock, lds, s>>>(a); \
    else if (stage == 2) k_scan<M, 2><<<grid, kScanBlock, lds, s>>>(a); \
    else k_scan<M, 3><<<grid, kScanBlock, lds, s>>>(a);                 \
  } while (0)
  if (mode == kModeLds) MSTX_SCAN(kModeLds);
  else if (mode == kModeDense) MSTX_SCAN(kModeDense);
  else if (mode == kModeBucket) MSTX_SCAN(kModeBucket);
  else MSTX_SCAN(kModeGlobal);
#undef MSTX_SCAN
  MSTX_LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_bucket_min(int round, int launched, const unsigned long long* offers,
                             const uint32_t* offT, int32_t nseg, const uint32_t* btot, unsigned long long* best,
                             const DevState* st, int grid, size_t lds, hipStream_t s) {
  k_bucket_min<<<grid, kScanBlock, lds + kBucketMinExtraLds, s>>>(round, launched, offers, offT, nseg, btot,
                                                                  best, st);
  MSTX_LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_slab_min(int round, int launched, int mode, const unsigned long long* slab, int64_t slab_cap,
                           int nwg, unsigned long long* best, unsigned long long* pbest, const DevState* st,
                           int grid, hipStream_t s) {
  const dim3 g2(grid, (nwg + kSlabRowsPerBlock - 1) / kSlabRowsPerBlock);
  k_slab_min<<<g2, kBlock, 0, s>>>(round, launched, mode, slab, slab_cap, nwg, best, pbest, st);
  MSTX_LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_dense_finish(int round, int launched, const unsigned long long* pbest, const uint32_t* seg_live,
                               int32_t nseg, const uint4* rec, uint8_t* in_mst, unsigned long long* total,
                               DevState* st, HostRound* host, hipStream_t s) {
  const int32_t kmax = launched_dense_limit(launched) < kDenseMax ? launched_dense_limit(launched) : kDenseMax;
  const size_t lds = dense_finish_lds(kmax);
  k_dense_finish<<<1, kDenseThreads, lds, s>>>(round, launched, pbest, seg_live, nseg, rec, in_mst, total, st, host);
  MSTX_LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_pair_collect(int round, int launched, const uint4* rec, const int32_t* labpool,
                               const uint32_t* seg_cnt, int32_t nseg, SparseTable sp, const DevState* st, int grid,
                               hipStream_t s) {
  k_pair_collect<<<grid, kBlock, 0, s>>>(round, launched, rec, labpool, seg_cnt, nseg, sp, st);
  MSTX_LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_sparse_finish(int round, int launched, const uint4* rec, SparseTable sp, const uint32_t* seg_live,
                                int32_t nseg, uint8_t* in_mst, unsigned long long* total, DevState* st,
                                HostRound* host, hipStream_t s) {
  k_sparse_finish<<<1, kSparseThreads, kMaxDynLds, s>>>(round, launched, rec, sp, seg_live, nseg, in_mst, total, st,
                                                        host);
  MSTX_LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_round_tail(int round, int32_t cap, const uint4* rec, unsigned long long* best, int32_t* parent,
                             int32_t* labpool, const uint32_t* seg_cnt, const uint32_t* seg_live, int32_t nseg,
                             uint8_t* in_mst, unsigned long long* total, uint32_t* btot, DevState* st,
                             HostRound* host, hipStream_t s) {
  const size_t lds = 8 * (size_t)(cap < 1 ? 1 : (cap > kTailMax ? kTailMax : cap));
  k_round_tail<<<1, kTailThreads, lds, s>>>(round, cap < kTailMax ? cap : kTailMax, rec, best, parent, labpool,
                                            seg_cnt, seg_live, nseg, in_mst, total, btot, st, host);
  MSTX_LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_hook(int round, const uint4* rec, const int32_t* labpool, const unsigned long long* best,
                       int32_t* parent, DevState* st, uint8_t* in_mst, uint32_t* part_sel,
                       unsigned long long* part_w, int grid, hipStream_t s) {
  k_hook<<<grid, kBlock, 0, s>>>(round, rec, labpool, best, parent, st, in_mst, part_sel, part_w);
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

hipError_t launch_finalize(int round, const int32_t* rootcnt, int32_t* rootpre, const uint32_t* seg_cnt,
                           const uint32_t* seg_live, int32_t nseg, const uint32_t* part_sel,
                           const unsigned long long* part_w, int32_t nhook, DevState* st,
                           unsigned long long* total, HostRound* host, hipStream_t s) {
  k_finalize<<<1, 1024, 0, s>>>(round, rootcnt, rootpre, seg_cnt, seg_live, nseg, part_sel, part_w, nhook, st,
                                total, host);
  MSTX_LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_relabel(int round, const int32_t* root_of, const unsigned long long* rootmask,
                          const int32_t* rootpre, int32_t* labpool, int32_t* parent, unsigned long long* best,
                          uint32_t* btot, const DevState* st, int grid, hipStream_t s) {
  k_relabel<<<grid, kBlock, 0, s>>>(round, root_of, rootmask, rootpre, labpool, parent, best, btot, st);
  MSTX_LAUNCH_CHECK();
  return hipSuccess;
}

}  // namespace mstx
