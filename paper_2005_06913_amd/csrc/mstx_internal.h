// mstx_internal.h -- declarations shared by the kernels and the host driver.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mstx {

// No edge: larger than every real key ((w << 32) | e, or the record position
// instead of e, both <= 0xFFFFFFFE).
static constexpr unsigned long long kKeyNone = ~0ull;

// Rounds recorded: components with an outgoing edge at least halve every
// round, so ceil(log2 n) + 1 <= 33 rounds for int32 n.
static constexpr int kMaxRounds = 40;

// Scan geometry: 1024-thread workgroups, 4 records per thread, one segment of
// the record stream = one tile = 4096 records.
static constexpr int kScanBlock = 1024;
static constexpr int kPerThread = 4;
static constexpr int kSegCap = kScanBlock * kPerThread;

// Ways of taking the per-component minima in the scan.
static constexpr int kModeGlobal = 0;  // filtered atomicMin on best[] in HBM
static constexpr int kModeLds = 1;     // per-workgroup minima in LDS, flushed once
static constexpr int kModeBucket = 2;  // offers sorted into component buckets + k_bucket_min
static constexpr int kModeDense = 3;   // last round: lightest edge per component pair, then finish
static constexpr int kNumModes = 4;

// gfx950 has 160 KiB of LDS per CU and gives all of it to one workgroup if
// asked; 1 KiB stays for the kernels' static LDS (at most 640 B today).
static constexpr int kMaxDynLds = 160 * 1024 - 1024;
static constexpr int32_t kLdsSlots = kMaxDynLds / 8;  // 20352 u64 minima
// Buckets hold at most 2^kMaxBucketShift = 16384 consecutive components (the
// LDS table of k_bucket_min), at most 1023 buckets (one counter per scan
// thread + total).
static constexpr int kMaxBuckets = 1023;
static constexpr int kMaxBucketShift = 14;
static constexpr int64_t kBucketMaxComponents = (int64_t)kMaxBuckets << kMaxBucketShift;
// Offer staging of one segment (2 offers per live edge).  With at most
// kOfferPadBuckets buckets every bucket's run is padded to a multiple of
// kOfferAlign offers, so each run of keys starts on a 128-byte line and the
// consumer fetches no line twice; the pad slots are written (whole lines)
// but never read.  A run is described by one word: start (bits 0..15) and
// length (bits 16..31).
static constexpr int kOfferAlign = 16;
static constexpr int kOfferPadBuckets = 256;
static constexpr int kOfferCap = 2 * kSegCap + kOfferAlign * kOfferPadBuckets;
static_assert(kOfferCap < (1 << 16) && 2 * kSegCap < (1 << 16), "offer run word");
// An offer is one word: the key's weight in bits 32..63, the key's low half
// minus the segment's first position (the edge's slot in its segment) in
// bits kOfferSlotShift.., and the component's index inside its bucket in the
// bits below.  The consumer knows the segment of every run, so it rebuilds
// the key exactly.
static constexpr int kOfferSlotShift = kMaxBucketShift;
static_assert(((uint64_t)(kSegCap - 1) << kOfferSlotShift) < (1ull << 32), "offer slot field");
// Bytes of dynamic LDS a BUCKET-mode scan uses: offer staging + counters.
static constexpr int kBucketScanLds = kOfferCap * 8 + (kMaxBuckets + 1) * 4;

// Buckets of width ceil(nr / 256) (at least 64, at most 16384): 256
// buckets, one k_bucket_min workgroup per CU, unless the width is at a
// bound.  Bucket of component c = c / width, by a multiply with a 32-bit
// reciprocal and one correction step (c < 2^24 here).
struct BucketGeom {
  int32_t width;
  int32_t nbk;
  uint32_t magic;  // floor((2^32 - 1) / width) + 1
};
__host__ __device__ inline BucketGeom bucket_geometry(int32_t nr) {
  int64_t wd = ((int64_t)nr + 255) / 256;
  if (wd < 64) wd = 64;
  if (wd > (1 << kMaxBucketShift)) wd = 1 << kMaxBucketShift;
  BucketGeom g;
  g.width = (int32_t)wd;
  g.nbk = (int32_t)(((int64_t)nr + wd - 1) / wd);
  g.magic = (uint32_t)(0xFFFFFFFFull / (uint64_t)wd + 1);
  return g;
}

// Dense finish: with at most kDenseMax components left, one pass over the live
// edges keeps the lightest edge of every component pair (any other edge
// between the same two components closes a cycle with a lighter one, so it is
// not in the tree), and one workgroup finishes Boruvka on that small complete
// graph with the pair table in LDS.  kDenseMax is the largest count whose
// table plus per-component state fits the dynamic LDS of one workgroup.
__host__ __device__ constexpr int32_t dense_pairs(int32_t k) { return k * (k - 1) / 2; }
__host__ __device__ constexpr size_t dense_finish_lds(int32_t k) {
  return (size_t)dense_pairs(k) * 8 + (size_t)k * 16;  // table; per group: key, added key, parent, target
}
static constexpr int32_t kDenseMax = 200;
static constexpr int32_t kDensePairsMax = dense_pairs(kDenseMax);
static_assert(dense_finish_lds(kDenseMax) <= (size_t)kMaxDynLds, "dense finish exceeds LDS");
static_assert(dense_finish_lds(kDenseMax + 1) > (size_t)kMaxDynLds, "kDenseMax is not the largest fit");
static_assert(kDensePairsMax <= kLdsSlots && kDenseMax < 256, "dense limit");
// Rounds with at most kTailMax components close in one workgroup
// (k_round_tail: hook, compress, finalize and relabel with the parent forest
// in LDS, 8 bytes per component, and ten components' edges per thread in
// registers).
static constexpr int32_t kTailMax = 10240;
// Sparse finish: a late round of at most kSparseMaxK components whose live
// edges join few distinct component pairs collects the lightest edge of every
// pair into a hash table of kSparseHash slots in the workspace (pair id,
// key; k_pair_collect) and, when they fit one workgroup's LDS as a small
// graph (sparse_pair_cap: 12 B per pair beside 18 B per component), finishes
// the solve there (k_sparse_finish); otherwise the round goes on as usual.
static constexpr int32_t kSparseMaxK = 8192;
static constexpr int kSparseHashBits = 15;
static constexpr int32_t kSparseHash = 1 << kSparseHashBits;
static constexpr int kSparseProbes = 64;  // a longer probe sequence counts as overflow
__host__ __device__ constexpr int32_t sparse_pair_cap(int32_t k) {
  return (int64_t)kMaxDynLds - 18 * (int64_t)k - 64 <= 0 ? 0
                                                          : (int32_t)(((int64_t)kMaxDynLds - 18 * (int64_t)k - 64) / 12);
}
static_assert(2 * sparse_pair_cap(0) <= kSparseHash, "hash load factor at most one half");
static_assert(kSparseMaxK <= kTailMax, "a round that tries the sparse finish can close in one workgroup");
// index of the unordered pair {a, b}, a < b < k, in row-major upper-triangle order
__host__ __device__ inline int32_t pair_index(int32_t a, int32_t b, int32_t k) {
  return a * k - a * (a + 1) / 2 + (b - a - 1);
}

// The `launched` word of a round: bit i = minima mode i was launched; bits
// 8..15 = the largest component count the dense finish takes (0: off).
__host__ __device__ inline int launched_dense_limit(int launched) { return (launched >> 8) & 0xFF; }

// Mode that handles n_r among the launched ones.
__host__ __device__ inline int pick_mode(int32_t nr, int launched) {
  if ((launched & (1 << kModeDense)) && nr <= launched_dense_limit(launched)) return kModeDense;
  if ((launched & (1 << kModeLds)) && nr <= kLdsSlots) return kModeLds;
  if ((launched & (1 << kModeBucket)) && (int64_t)nr <= kBucketMaxComponents) return kModeBucket;
  return kModeGlobal;
}

// Record formats of the edge stream (rounds >= 1).  A wide record is
// {a, b, w, e} in 16 bytes.  Once a round's labels fit 16 bits (n_r <=
// kNarrowMax) its survivors are written as narrow records, a | b << 16 | w <<
// 32 in 8 bytes, with e stored apart: segment s (kSegCap records) keeps its
// narrow records in the first 32 KB of its 64 KB wide area and their edge
// indices in the next 16 KB, so an in-place rewrite never leaves the segment.
static constexpr int32_t kNarrowMax = 65536;
__host__ __device__ constexpr uint64_t narrow_rec_index(uint32_t pos) {
  return (uint64_t)pos + (uint64_t)(pos & ~(uint32_t)(kSegCap - 1));  // u64 index
}
__host__ __device__ constexpr uint64_t narrow_e_index(uint32_t pos) {
  return 4 * (uint64_t)(pos & ~(uint32_t)(kSegCap - 1)) + 2 * kSegCap + (pos & (kSegCap - 1));  // u32 index
}
// Records a round reads: 0 the caller's arrays (round 0), 1 the caller's
// arrays through round 0's labels (round 1), 2 wide records, 3 narrow records.
// Round q >= 2 reads narrow records iff n_{q-1} <= kNarrowMax.
__host__ __device__ constexpr int scan_stage(int q, int64_t n_prev) {
  return q == 0 ? 0 : (q == 1 ? 1 : (n_prev <= kNarrowMax ? 3 : 2));
}
// What a round that reads narrow records does with them (DevState::keep):
// kMoveRecords compacts the survivors (the default, and always when at least
// 1/kKeepDeadDen of the records the previous round read were dead there);
// otherwise kKeepRecords leaves them untouched when the composed label map
// the round after it then reads (two buffers of kNarrowMax entries, used
// alternately) can still be staged in that round's LDS, and
// kRelabelRecords rewrites every record's labels in place (same positions,
// no edge-index traffic) when it cannot.
static constexpr int kKeepDeadDen = 4;
static constexpr int kMoveRecords = 0;
static constexpr int kKeepRecords = 1;
static constexpr int kRelabelRecords = 2;

// Minima modes launched for a round whose component count is at most
// `bound` (exact: it is the count), reading stream `stage`; bit i = mode i.
// Besides the mode of the bound itself, the LDS mode is launched whenever a
// 64-fold drop (8-fold in round 1) would bring the count into its range, and
// the dense mode whenever an 8-fold drop would: a launch that finds another
// mode chosen returns at once.
__host__ __device__ inline int scan_modes(int64_t bound, bool exact, int stage, int dense_limit, bool buckets,
                                          int64_t bucket_limit) {
  const int64_t blim = buckets ? bucket_limit : 0;
  const int hi = bound <= dense_limit ? kModeDense
                 : bound <= kLdsSlots ? kModeLds
                 : bound <= blim      ? kModeBucket
                                      : kModeGlobal;
  int mask = 1 << hi;
  if (!exact) {
    if (hi != kModeDense && dense_limit > 0 && bound / 8 <= dense_limit) mask |= 1 << kModeDense;
    const int64_t drop = stage == 1 ? 8 : 64;
    if (hi != kModeLds && hi != kModeDense && bound / drop <= kLdsSlots) mask |= 1 << kModeLds;
    if (hi == kModeGlobal && buckets && bound / 8 <= bucket_limit) mask |= 1 << kModeBucket;
  }
  if (!buckets) {
    mask &= ~(1 << kModeBucket);
    if (bound > kLdsSlots) mask |= 1 << kModeGlobal;
  }
  return mask;
}
// Dynamic LDS of the minima table of an LDS or dense launch for `bound`.
__host__ __device__ inline int64_t scan_table_lds(int mode, int64_t bound, int dense_limit) {
  if (mode == kModeDense) {
    const int64_t k = bound < 2 ? 2 : (bound < dense_limit ? bound : dense_limit);
    return (int64_t)dense_pairs((int32_t)k) * 8;
  }
  const int64_t slots = bound < 1 ? 1 : (bound < kLdsSlots ? bound : kLdsSlots);
  return slots * 8;
}
// Whether an LDS or dense launch for `bound` can stage a label map of `dom`
// entries behind its table (2 bytes each, 1 in dense mode).
__host__ __device__ inline bool map_fits_lds(int mode, int64_t bound, int dense_limit, int64_t dom) {
  const int64_t off = (scan_table_lds(mode, bound, dense_limit) + 15) & ~(int64_t)15;
  return off + (mode == kModeDense ? 1 : 2) * dom <= (int64_t)kMaxDynLds;
}

// Device-resident round state.  Round r's kernels read n[r], lab_off[r],
// keep[r], map_off[r] and map_n[r]; the finalize kernel of round r writes
// n[r+1], lab_off[r+1], live[r], sel[r], stream[r+1], keep[r+1], map_off[r+1]
// and map_n[r+1].
struct DevState {
  int32_t n[kMaxRounds + 2];        // components entering round r (isolated ones dropped)
  int64_t lab_off[kMaxRounds + 2];  // offset of round r's label map in the label pool
  int64_t live[kMaxRounds + 1];     // edges between different components at round r
  int64_t sel[kMaxRounds + 1];      // edges added in round r
  int64_t stream[kMaxRounds + 2];   // records (or input edges) round r reads
  int64_t map_off[kMaxRounds + 2];  // label-pool offset of the map from record labels to round r's
  int32_t map_n[kMaxRounds + 2];    // ... and its entries
  int32_t keep[kMaxRounds + 2];     // what round r does with the records it reads (kMoveRecords ..)
  int64_t edges_added;              // running total of sel[]
  int64_t m;                        // input edges
  int64_t cmap_off;                 // label-pool offset of the two composed-map buffers
  int32_t dense_limit;              // the dense finish's component limit of this solve (0: off)
  int32_t err;                      // an edge end outside [0, n) was seen
  int32_t err_internal;             // a label lookup gave an impossible value
  int32_t dense_at;                 // round that ended with the dense finish (-1: none)
  int32_t pad;
};

// What the finalize kernel of round r writes to pinned host memory.
struct HostRound {
  int32_t n_next;
  int32_t err;
  int32_t err_internal;
  int32_t dense;  // 1: the dense finish ended the solve in this round, 2: the sparse finish
  int64_t live;
  int64_t sel;
  int64_t edges_added;
  int64_t stream;  // records (or input edges) the round read
  int32_t map_n;      // entries of the label map the round read
  int32_t keep;       // what the round did with its records (kMoveRecords ..)
  int32_t keep_next;  // ... and what the next round does
  int32_t pad;
};

// Arguments of the scan kernel (passed by value).
struct ScanArgs {
  int round;
  int launched;  // bit mask of the modes launched for this round
  const int32_t* src;
  const int32_t* dst;
  const uint32_t* w;
  uint32_t m;
  int32_t n;
  const int32_t* labpool;
  uint4* rec;
  uint32_t* seg_cnt;   // records per segment (written when the round rewrites them)
  uint32_t* seg_live;  // live records per segment this round
  int32_t nseg;
  unsigned long long* best;
  DevState* st;
  unsigned long long* offers;   // BUCKET mode offers: [nseg][kOfferCap]
  uint32_t* offT;               // [kMaxBuckets + 1][nseg] run starts
  unsigned long long* slab;     // LDS mode, n_r > kSlabMin: per-workgroup minima [grid][n_r]
  int64_t slab_cap;             // entries of slab
  unsigned long long* pbest;    // dense mode: lightest key per component pair [kDensePairsMax]
  int32_t lds_bytes;            // dynamic LDS of the launch (LDS / DENSE mode: the table for n_r,
                                // then the first entries of the label map that fit, rounds >= 2)
  uint32_t* btot;               // BUCKET mode: offers per bucket, summed over the scan [kMaxBuckets]
  const uint8_t* in_mst;        // round 1: the edges round 0 added (dead now), or null
};

// LDS-mode minima of more than kSlabMin components are flushed through a
// per-workgroup slab and a column minimum (k_slab_min) instead of atomics --
// unless the round's stream is short next to the rows: a record lowers at
// most two minima, so a workgroup's atomics are at most twice its records,
// while its row is all n_r entries (written, then read again).  With
// `stream` records and nwg rows the atomics win below about nwg * n_r /
// kSlabStreamRatio records (an atomic merge costs about twice the traffic
// of a row entry).  Dense mode passes no stream (always the slab).
static constexpr int32_t kSlabMin = 512;
static constexpr int64_t kSlabStreamRatio = 4;
static constexpr int64_t kSlabAnyStream = (int64_t)1 << 60;
__host__ __device__ inline bool use_slab(const unsigned long long* slab, int64_t cap, int32_t nr, int nwg,
                                         int64_t stream) {
  return slab != nullptr && nr > kSlabMin && (int64_t)nwg * nr <= cap &&
         kSlabStreamRatio * stream >= (int64_t)nwg * nr;
}

// Batched solve: graphs with at most kSmallN vertices are solved by one
// workgroup each with the vertex state in LDS (best u64 + comp + parents).
static constexpr int32_t kSmallN = 8192;
// A single graph (mst_solve) with at most the small-graph limit of vertices
// (kSmallN by default, see mst_set_small_limit) and at most kSmallMaxEdges
// edges is solved the same way: one launch instead of a chain per round.
static constexpr int64_t kSmallMaxEdges = 1 << 17;
static constexpr int kSmallStatsWords = 1 + 3 * (kMaxRounds + 1);
static constexpr int kSmallSolveLds = kSmallN * (8 + 4 + 4);
// Whether the one-workgroup small solve keeps a graph's edges (12 B each) in
// LDS behind its vertex state (16 B per vertex) in the batched launch.
__host__ __device__ constexpr bool small_edges_cached(int64_t n, int64_t m) {
  return ((16 * n + 15) & ~(int64_t)15) + 12 * m <= (int64_t)kMaxDynLds;
}
// Batched solve: graphs with kSmallN < n <= kMidN vertices (default; see
// mst_set_mid_limit) and at most kMidMaxEdges edges are solved by one
// workgroup each as well, with 10 bytes of LDS per vertex: the minimum key
// (u64) and a 2-byte union-find.
static constexpr int32_t kMidN = 16280;
static constexpr int64_t kMidMaxEdges = 1 << 21;
__host__ __device__ constexpr size_t mid_solve_lds(int32_t n) {
  return (size_t)8 * (size_t)n + (((size_t)2 * (size_t)n + 3) & ~(size_t)3);
}
static_assert(mid_solve_lds(kMidN) <= (size_t)kMaxDynLds, "the mid-size layout fits the LDS allocation");

hipError_t configure_kernels();
hipError_t configure_batched_kernels();
// Arguments of the mid-size solve: graphs glist[i] of the batch (voff, eoff,
// src, dst, w as the caller gave them), or, when contracted, the same graphs
// after their first rounds (pre_contract_body): nlist[i] components left, both ends of local
// edge j as 16-bit component numbers in pairs[poff[i] + j], pcnt[i] edges and
// their weight (in total[g]) taken by the contraction rounds, pbad[i] set when the
// graph had out-of-range ids, max_n the launch's bound on nlist.
struct MidArgs {
  const int32_t* glist;
  const int64_t* voff;
  const int64_t* eoff;
  const int32_t* src;
  const int32_t* dst;
  const uint32_t* w;
  const uint32_t* pairs;
  const int64_t* poff;
  const int32_t* nlist;
  const int32_t* pcnt;
  const int32_t* pbad;
  uint8_t* in_mst;
  unsigned long long* total;
  int32_t* status;
  int32_t max_n;
};
// Arguments of the contraction of graphs glist[i] (n <= kPreMaxN) by their
// first rounds until at most `target` components are left: scratch from
// element soff[i] holds n u64; the outputs (pairs, nlist, pcnt, pbad, total,
// in_mst) are those MidArgs describes for the contracted solve.
static constexpr int32_t kPreMaxN = 65536;
struct PreArgs {
  const int32_t* glist;
  const int64_t* voff;
  const int64_t* eoff;
  const int32_t* src;
  const int32_t* dst;
  const uint32_t* w;
  const int64_t* soff;
  unsigned long long* scratch;
  uint32_t* pairs;
  const int64_t* poff;
  int32_t* nlist;
  int32_t* pcnt;
  int32_t* pbad;
  uint8_t* in_mst;
  unsigned long long* total;
  int32_t target;
};
// One launch for every graph of a batch solved by one workgroup: ncon
// contracted (pre, then con), nmid mid-size (mid), nsmall small (small's
// glist, voff, eoff, src, dst, w, in_mst, total, status).
struct BatchSolveArgs {
  PreArgs pre;
  MidArgs con;
  MidArgs mid;
  MidArgs small;
  int32_t ncon;
  int32_t nmid;
};
hipError_t launch_batch_solve(const BatchSolveArgs& B, int nsmall, hipStream_t s);
// Edge list of a symmetric CSR adjacency (mstx_csr.hip): csr_tiles(nnz) tile
// counts (cnt), their exclusive scan plus the total (off, csr_tiles + 1), an
// error word (bit 0: row_ptr, bit 1: a column outside [0, n)) the caller zeroes.
int64_t csr_tiles(int64_t nnz);
hipError_t launch_csr_to_edges(int32_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col, const uint32_t* w,
                               uint32_t* cnt, int64_t* off, uint32_t* err, int32_t* out_src, int32_t* out_dst,
                               uint32_t* out_w, hipStream_t s);
hipError_t launch_small_solve_single(int32_t n, int64_t m, const int32_t* src, const int32_t* dst,
                                     const uint32_t* w, uint8_t* in_mst, unsigned long long* total,
                                     int32_t* status, int64_t* stats, hipStream_t s);
hipError_t launch_gather(const int32_t* glist, int ng, const int64_t* voff, const int64_t* eoff,
                         const int64_t* cvert, const int64_t* cedge, int64_t chunk_edges, const int32_t* src,
                         const int32_t* dst, const uint32_t* w, int32_t* gsrc, int32_t* gdst, uint32_t* gw,
                         int32_t* gbad, hipStream_t s);
hipError_t launch_graph_epilogue(const int32_t* glist, int ng, const int64_t* voff, const int64_t* eoff,
                                 const int64_t* cedge, int64_t max_graph_m, const uint8_t* cin_mst,
                                 const uint32_t* gw, const int32_t* gbad, uint8_t* in_mst,
                                 unsigned long long* acc_w, uint32_t* acc_c, unsigned long long* total,
                                 int32_t* status, hipStream_t s);
// The sparse finish's pair table in the workspace (all null: none).
struct SparseTable {
  uint32_t* pid;            // [kSparseHash] lo * n_r + hi of the pair held, kPairEmpty: free
  unsigned long long* key;  // [kSparseHash] lightest key of that pair
  uint32_t* state;          // [0] slots claimed, [1] overflow
};
static constexpr uint32_t kPairEmpty = 0xFFFFFFFFu;

hipError_t launch_init(int32_t n, int64_t m, int64_t cmap_off, int dense_limit, unsigned long long* best,
                       int32_t* parent, unsigned long long* pbest, uint32_t* btot, SparseTable sp, DevState* st,
                       int grid, hipStream_t s);
hipError_t launch_pair_collect(int round, int launched, const uint4* rec, const int32_t* labpool,
                               const uint32_t* seg_cnt, int32_t nseg, SparseTable sp, const DevState* st, int grid,
                               hipStream_t s);
hipError_t launch_sparse_finish(int round, int launched, const uint4* rec, SparseTable sp, const uint32_t* seg_live,
                                int32_t nseg, uint8_t* in_mst, unsigned long long* total, DevState* st,
                                HostRound* host, hipStream_t s);
hipError_t launch_fill_u8(uint8_t* p, int64_t count, uint8_t v, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long* p, int64_t count, unsigned long long v, int grid,
                           hipStream_t s);
hipError_t launch_scan(int mode, int stage, const ScanArgs& a, int grid, size_t lds, hipStream_t s);
hipError_t launch_bucket_min(int round, int launched, const unsigned long long* offers, const uint32_t* offT,
                             int32_t nseg, const uint32_t* btot, unsigned long long* best, const DevState* st, int grid,
                             size_t lds, hipStream_t s);
hipError_t launch_slab_min(int round, int launched, int mode, const unsigned long long* slab, int64_t slab_cap,
                           int nwg, unsigned long long* best, unsigned long long* pbest, const DevState* st,
                           int grid, hipStream_t s);
hipError_t launch_dense_finish(int round, int launched, const unsigned long long* pbest, const uint32_t* seg_live,
                               int32_t nseg, const uint4* rec, uint8_t* in_mst, unsigned long long* total,
                               DevState* st, HostRound* host, hipStream_t s);
hipError_t launch_hook(int round, const uint4* rec, const int32_t* labpool, const unsigned long long* best,
                       int32_t* parent, DevState* st, uint8_t* in_mst, uint32_t* part_sel,
                       unsigned long long* part_w, int grid, hipStream_t s);
hipError_t launch_compress(int round, int32_t* parent, int32_t* root_of, const unsigned long long* best,
                           unsigned long long* rootmask, int32_t* rootcnt, const DevState* st, int grid,
                           hipStream_t s);
hipError_t launch_round_tail(int round, int32_t cap, const uint4* rec, unsigned long long* best, int32_t* parent,
                             int32_t* labpool, const uint32_t* seg_cnt, const uint32_t* seg_live, int32_t nseg,
                             uint8_t* in_mst, unsigned long long* total, uint32_t* btot, DevState* st,
                             HostRound* host, hipStream_t s);
hipError_t launch_finalize(int round, const int32_t* rootcnt, int32_t* rootpre, const uint32_t* seg_cnt,
                           const uint32_t* seg_live, int32_t nseg, const uint32_t* part_sel,
                           const unsigned long long* part_w, int32_t nhook, DevState* st,
                           unsigned long long* total, HostRound* host, hipStream_t s);
hipError_t launch_relabel(int round, const int32_t* root_of, const unsigned long long* rootmask,
                          const int32_t* rootpre, int32_t* labpool, int32_t* parent, unsigned long long* best,
                          uint32_t* btot, const DevState* st, int grid, hipStream_t s);

}  // namespace mstx
