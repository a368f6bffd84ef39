// mstx_host.hip -- host driver and C ABI of the parallel Boruvka MST.
//
// Argument checks run on the host before any HIP call.  The workspace (all
// device scratch) is planned from (n, m), cached per device and guarded by a
// mutex.
//
// Round control is pipelined one round ahead: round r+1 is enqueued before
// the host waits for round r's record (written by k_finalize straight into
// pinned host memory), so the GPU never idles on the host.  When round r+1
// is enqueued only an upper bound n_{r+1} <= n_r / 2 is known; the scan
// modes are launched for every count the bound allows and the kernels pick
// the one that matches the actual count on the device (the others return
// at once).  The round after the last one finds n <= 1 and returns at once.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <utility>
#include <vector>

#include "mstx.h"
#include "mstx_internal.h"

// Device scratch of mst_solve_noalloc, for callers that cannot allocate: the
// workspace of one solve, its round records and the one-workgroup path's
// status words.  Each device the library runs on holds its own copy (the
// code object's data segment) until the process ends.  In host code this
// name is only a handle: its device address comes from hipGetSymbolAddress,
// once per device.
static constexpr size_t kNoAllocScratchBytes = size_t(256) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace mstx {
namespace {

constexpr int kBlockThreads = 256;
constexpr int kMaxGrid = 4096;  // capacity of the per-block partial arrays (hook)

struct Layout {
  size_t best, parent, root_of, labpool, cmap, rootmask, rootcnt, rootpre, rec, seg_cnt, seg_live, part_sel,
      part_w, state, pbest, btot, sp_pid, sp_key, sp_state, offers, offT, slab, bytes;
  int64_t slab_cap;  // u64 entries of the LDS-mode slab (0: none)
  int32_t nseg;
  bool bucket;  // offer buffers present
};

constexpr int kSlabRows = 256;  // workgroup rows of the LDS-mode slab

constexpr size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

// Workspace plan for a graph with n vertices and m edges.
Layout plan(int32_t n, int64_t m) {
  Layout L{};
  const size_t N = (size_t)std::max<int32_t>(n, 1);
  const size_t words = (N + 63) / 64 + 1;
  const int64_t nseg = std::max<int64_t>(1, (m + kSegCap - 1) / kSegCap);
  L.nseg = (int32_t)nseg;
  L.bucket = n > kLdsSlots;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  L.best = take(8 * N);
  L.parent = take(4 * N);
  L.root_of = take(4 * N);
  L.labpool = take(4 * (2 * N + 64));  // label maps: n_0 + n_1 + ... < 2n
  L.cmap = take(4 * 2 * (size_t)kNarrowMax);  // composed maps of rounds that keep their records
  L.rootmask = take(8 * words);
  L.rootcnt = take(4 * words);
  L.rootpre = take(4 * words);
  L.rec = take(16 * (size_t)nseg * kSegCap);
  L.seg_cnt = take(4 * (size_t)nseg);
  L.seg_live = take(4 * (size_t)nseg);
  L.part_sel = take(4 * (size_t)kMaxGrid);
  L.part_w = take(8 * (size_t)kMaxGrid);
  L.state = take(sizeof(DevState));
  L.pbest = take(8 * (size_t)kDensePairsMax);
  L.btot = take(4 * (size_t)kMaxBuckets);
  L.sp_pid = take(4 * (size_t)kSparseHash);  // the sparse finish's pair table
  L.sp_key = take(8 * (size_t)kSparseHash);
  L.sp_state = take(16);
  L.slab_cap = n > kSlabMin ? (int64_t)kSlabRows * std::min<int32_t>(n, kLdsSlots) : 0;
  if (L.slab_cap) L.slab = take(8 * (size_t)L.slab_cap);
  if (L.bucket) {
    L.offers = take(8 * (size_t)nseg * kOfferCap);
    L.offT = take(4 * (size_t)(kMaxBuckets + 1) * nseg);
  }
  L.bytes = off;
  return L;
}

struct DeviceCache {
  std::mutex mu;
  void* base = nullptr;
  size_t bytes = 0;
  HostRound* host_rounds = nullptr;  // pinned, one record per round
  hipEvent_t round_ev[kMaxRounds + 1] = {};
  int cus = 0;
  bool configured = false;
  void* aux = nullptr;  // batched-call scratch
  size_t aux_bytes = 0;
  void* small_dev = nullptr;       // single small graph: status + round statistics
  int64_t* small_host = nullptr;   // pinned copy of the same
  // the stepwise solve of this stream (mst_solve_begin): its own workspace,
  // records and events, so calls on the stream may run between its rounds
  void* step_base = nullptr;
  size_t step_bytes = 0;
  HostRound* step_rounds = nullptr;
  hipEvent_t step_ev[kMaxRounds + 1] = {};
  bool step_active = false;
};

// One cache per (device, stream): calls on different streams have their own
// workspace and run concurrently; calls on the same stream are serialised.
std::mutex g_caches_mu;

// Largest component count the dense finish takes (0: every round is a plain
// Boruvka round); mst_set_dense_limit() changes it.
std::atomic<int> g_dense_limit{kDenseMax};
// Largest vertex count for which mst_solve takes the one-workgroup path
// (0: never); mst_set_small_limit() changes it.
std::atomic<int> g_small_limit{kSmallN};
// Largest vertex count for which mst_solve_batched solves a graph above
// kSmallN vertices with one workgroup (the mid-size solve) instead of the union
// chunks (0: never); mst_set_mid_limit() changes it.
std::atomic<int> g_mid_limit{kMidN};
// Largest component-count bound for which a round's hook .. relabel run as
// one workgroup (0: never); mst_set_tail_limit() changes it.
std::atomic<int> g_tail_limit{kTailMax};
// Largest component-count bound for which a round's scan takes its minima in
// bucket mode; above it (and above the LDS range) the filtered global atomics
// of GLOBAL mode.  mst_set_bucket_limit() changes it.
std::atomic<int64_t> g_bucket_limit{kBucketMaxComponents};
// Workgroups per CU of an LDS-mode scan (0: chosen from its LDS size, at
// most 4; else this many as far as 160 KB of LDS per CU holds them);
// mst_set_scan_occupancy() changes it.
std::atomic<int> g_scan_occupancy{0};
// The sparse finish is tried in a round whose bound on the component count
// is at most kSparseMaxK when at most this many live edges were left two
// rounds before (0: never); mst_set_sparse_limit() changes it.
constexpr int32_t kSparseLiveDefault = 1 << 20;
std::atomic<int> g_sparse_limit{kSparseLiveDefault};
std::map<std::pair<int, hipStream_t>, std::unique_ptr<DeviceCache>> g_caches;

// Per-round statistics of the calling thread's last single-graph solve
// (components, live edges, edges added per round), in a fixed-size array.
struct RoundStats {
  int rounds = 0;
  int64_t v[3 * (kMaxRounds + 1)] = {};
  void clear() { rounds = 0; }
};
thread_local RoundStats t_last_stats;

size_t workspace_limit() {
  const char* s = std::getenv("MSTX_WORKSPACE_LIMIT_BYTES");
  if (!s || !*s) return SIZE_MAX;
  char* end = nullptr;
  const unsigned long long v = std::strtoull(s, &end, 10);
  return (end && *end == 0) ? (size_t)v : SIZE_MAX;
}

int grid_for(int64_t items, int per_block = kBlockThreads, int cap = kMaxGrid) {
  const int64_t g = (items + per_block - 1) / per_block;
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, cap));
}

// Host-only argument validation shared by the entry points.
int check_args(int32_t n, int64_t m, const void* src, const void* dst, const void* w) {
  if (n < 0 || m < 0) return MSTX_ERR_INVALID_ARG;
  if (m > (int64_t)0xFFFFFFFFLL) return MSTX_ERR_TOO_LARGE;
  if (m > 0 && (!src || !dst || !w)) return MSTX_ERR_INVALID_ARG;
  return MSTX_OK;
}

#define HIP_OK(expr)                                  \
  do {                                                \
    if ((expr) != hipSuccess) return MSTX_ERR_DEVICE; \
  } while (0)

// Locks the cache of (current device, stream), grows its workspace to `bytes`.
int acquire(DeviceCache*& dc, std::unique_lock<std::mutex>& lock, size_t bytes, hipStream_t stream) {
  int dev = 0;
  HIP_OK(hipGetDevice(&dev));
  {
    std::lock_guard<std::mutex> g(g_caches_mu);
    auto& slot = g_caches[{dev, stream}];
    if (!slot) slot.reset(new DeviceCache());
    dc = slot.get();
  }
  lock = std::unique_lock<std::mutex>(dc->mu);
  if (!dc->configured) {
    HIP_OK(hipHostMalloc((void**)&dc->host_rounds, sizeof(HostRound) * (kMaxRounds + 1), hipHostMallocDefault));
    // The round events carry no system-scope fence (a cache write-back per
    // round): the kernel that writes a round's record publishes it itself
    // with a system-scope fence, and the host checks that it is there.
    for (int i = 0; i <= kMaxRounds; ++i)
      HIP_OK(hipEventCreateWithFlags(&dc->round_ev[i], hipEventDisableTiming | hipEventDisableSystemFence));
    hipDeviceProp_t prop;
    HIP_OK(hipGetDeviceProperties(&prop, dev));
    dc->cus = prop.multiProcessorCount;
    // raises the dynamic LDS limit of the scan kernels; if the runtime refuses,
    // launches that need more LDS fail and report MSTX_ERR_DEVICE
    if (configure_kernels() != hipSuccess) (void)hipGetLastError();
    if (configure_batched_kernels() != hipSuccess) (void)hipGetLastError();
    dc->configured = true;
  }
  if (bytes > 0 && dc->bytes < bytes) {
    // stream-ordered: only this stream uses the workspace, so growing it
    // waits for this stream's earlier work and for no other stream's
    if (dc->base) {
      HIP_OK(hipFreeAsync(dc->base, stream));
      dc->base = nullptr;
      dc->bytes = 0;
    }
    if (hipMallocAsync(&dc->base, bytes, stream) != hipSuccess) {
      (void)hipGetLastError();
      dc->base = nullptr;
      return MSTX_ERR_OUT_OF_MEMORY;
    }
    dc->bytes = bytes;
  }
  return MSTX_OK;
}

template <typename T>
T* at(void* base, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(base) + off);
}

int rounds_bound(int32_t n) {
  int b = 0;
  while (b < 31 && (1LL << b) < (long long)n) ++b;
  return b + 1;
}

// ------------------------------------------------------------- profiling
// Opt-in per-kernel timing: when enabled, every kernel launch of a solve is
// bracketed by two hipEvents on the solve's stream.  After the solve the
// elapsed times are accumulated per kernel (template instantiation, as a
// profiler lists them), every launch counted -- also those that returned at
// once (a minima mode not chosen for the actual count, the round enqueued
// after the last one).  The scan launch that did a round's work is credited
// with the round's algorithmic bytes (what the method must move, from the
// round statistics).
enum Kind {
  kScanFirst = 0,  // 4 stages x 4 minima modes: kind = kNumModes * stage + mode
  kBucketMin = 16, kSlabMin_, kDenseFinish, kHook, kCompress, kFinalize, kRelabel, kSmallSolve, kRoundTail,
  kPairCollect, kSparseFinish, kKinds
};
constexpr int kScanKinds = 16;
// Names as rocprofv3 reports the kernels (template arguments: minima mode
// 0 global / 1 LDS / 2 bucket / 3 dense; the stream read: 0 the caller's
// edges, 1 the caller's edges through round 0's labels, 2 wide records,
// 3 narrow records).
const char* const kKindNames[kKinds] = {
    "k_scan<0, 0>", "k_scan<1, 0>", "k_scan<2, 0>", "k_scan<3, 0>",
    "k_scan<0, 1>", "k_scan<1, 1>", "k_scan<2, 1>", "k_scan<3, 1>",
    "k_scan<0, 2>", "k_scan<1, 2>", "k_scan<2, 2>", "k_scan<3, 2>",
    "k_scan<0, 3>", "k_scan<1, 3>", "k_scan<2, 3>", "k_scan<3, 3>",
    "k_bucket_min", "k_slab_min", "k_dense_finish", "k_hook", "k_compress", "k_finalize", "k_relabel",
    "k_small_solve", "k_round_tail", "k_pair_collect", "k_sparse_finish"};

int scan_kind(int stage, int mode) { return kNumModes * stage + mode; }

struct Profile {
  std::mutex mu;
  bool enabled = false;
  double ms[kKinds] = {};
  int64_t launches[kKinds] = {};
  double bytes[kKinds] = {};
  // the same per round of the solve (round index as the launch was enqueued)
  double rms[kMaxRounds + 1][kKinds] = {};
  int64_t rlaunches[kMaxRounds + 1][kKinds] = {};
  double rbytes[kMaxRounds + 1][kKinds] = {};
  void clear() {
    for (int k = 0; k < kKinds; ++k) {
      ms[k] = bytes[k] = 0.0;
      launches[k] = 0;
      for (int r = 0; r <= kMaxRounds; ++r) {
        rms[r][k] = rbytes[r][k] = 0.0;
        rlaunches[r][k] = 0;
      }
    }
  }
};
Profile g_prof;

struct PendingLaunch {
  int kind, round, mode;  // mode: -1 for kernels that always run
  hipEvent_t a, b;
};

struct LaunchTimer {
  bool on = false;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  std::vector<PendingLaunch> pending;
  hipStream_t s = nullptr;

  void begin(hipStream_t stream) {
    {
      std::lock_guard<std::mutex> g(g_prof.mu);
      on = g_prof.enabled;
    }
    used = 0;
    pending.clear();
    s = stream;
  }
  hipEvent_t event() {
    if (used == pool.size()) {
      hipEvent_t e = nullptr;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      pool.push_back(e);
    }
    return pool[used++];
  }
  int start(int kind, int round, int mode) {
    if (!on) return -1;
    PendingLaunch p{kind, round, mode, event(), event()};
    if (!p.a || !p.b || hipEventRecord(p.a, s) != hipSuccess) return -1;
    pending.push_back(p);
    return (int)pending.size() - 1;
  }
  void stop(int slot) {
    if (slot >= 0) (void)hipEventRecord(pending[slot].b, s);
  }
  // After the stream is synchronised.  chosen[r] = mode that ran in round r,
  // bytes[r] = algorithmic bytes of round r's scan, bmin[r] those of its
  // bucket minima, other[r][kind] those of the round's other kernels (the
  // mode-bound ones count when their mode ran); rounds >= nrounds were idle.
  void commit(int nrounds, const int* chosen, const double* bytes, const double* bmin,
              const double (*other)[kKinds]) {
    if (!on) return;
    std::lock_guard<std::mutex> g(g_prof.mu);
    for (const auto& p : pending) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, p.a, p.b) != hipSuccess) continue;
      double b = 0.0;
      if (p.round >= 0 && p.round < nrounds) {
        const bool moded = p.kind < kScanKinds || p.kind == kBucketMin || p.kind == kSlabMin_ || p.kind == kDenseFinish;
        if (!moded) b = other[p.round][p.kind];
        else if (p.mode == chosen[p.round])
          b = p.kind < kScanKinds ? bytes[p.round] : (p.kind == kBucketMin ? bmin[p.round] : other[p.round][p.kind]);
      }
      g_prof.ms[p.kind] += ms;
      g_prof.launches[p.kind] += 1;
      g_prof.bytes[p.kind] += b;
      const int r = p.round < 0 ? 0 : (p.round > kMaxRounds ? kMaxRounds : p.round);
      g_prof.rms[r][p.kind] += ms;
      g_prof.rlaunches[r][p.kind] += 1;
      g_prof.rbytes[r][p.kind] += b;
    }
    pending.clear();
  }
};
thread_local LaunchTimer t_timer;

// Everything one solve needs to enqueue its rounds.
struct Solve {
  int32_t n;
  int64_t m;
  const int32_t* src;
  const int32_t* dst;
  const uint32_t* w;
  uint8_t* in_mst;
  unsigned long long* total;
  hipStream_t s;
  int cus;               // compute units of the device
  HostRound* rounds;     // round records: pinned host memory, or device memory
  hipEvent_t* events;    // one event per round, recorded after it (nullptr: none)
  Layout L;
  unsigned long long* best;
  int32_t* parent;
  int32_t* root_of;
  int32_t* labpool;
  unsigned long long* rootmask;
  int32_t* rootcnt;
  int32_t* rootpre;
  uint4* rec;
  uint32_t* seg_cnt;
  uint32_t* seg_live;
  uint32_t* part_sel;
  unsigned long long* part_w;
  DevState* st;
  unsigned long long* offers;
  uint32_t* offT;
  unsigned long long* slab;
  unsigned long long* pbest;
  uint32_t* btot;
  SparseTable sp;
  int dense_limit;            // 0: no dense finish
  int64_t sparse_limit;       // live-edge bound below which the sparse finish is tried (0: never)
  int64_t live_rec[kMaxRounds + 1];  // live edges of round r, from its record (taken before round r + 2 is enqueued)
  bool sparse_tried[kMaxRounds + 1];
  int tail_limit;             // 0: every round takes the multi-workgroup hook .. relabel
  int64_t bucket_limit;       // largest bound that may take bucket mode (0: never)
  int launched[kMaxRounds + 1];  // per round
  int stage[kMaxRounds + 1];     // the stream each enqueued round reads (scan_stage)
  int64_t dom[kMaxRounds + 1];   // entries of its label map
  int keep[kMaxRounds + 2];      // round r keeps its records in place (from round r - 1's record)
};

// Enqueues the scan of round r reading stream `stage` (scan_stage) whose
// component count is at most `bound`; `dom` bounds the entries of the round's
// label map.  Returns the launched mask.
int enqueue_scan(Solve& S, int r, int stage, int64_t bound, bool exact, hipError_t& err, int64_t dom = 0) {
  LaunchTimer& T = t_timer;
  const bool buckets = S.L.bucket && S.bucket_limit > 0;
  // the actual count may be much smaller than the bound: a skewed graph can
  // lose far more than half its components in a round.  Round 1 is covered
  // for an 8-fold drop only: on random and grid graphs the first round leaves
  // about a quarter of the vertices and the extra launch would return every
  // time; a graph that falls further still takes bucket mode, correct, for
  // that one round
  int launched = scan_modes(bound, exact, stage, S.dense_limit, buckets, S.bucket_limit);
  launched |= S.dense_limit << 8;
  ScanArgs A{r,         launched,   S.src,    S.dst,  S.w,      (uint32_t)S.m, S.n,      S.labpool,
             S.rec,     S.seg_cnt,  S.seg_live, S.L.nseg, S.best, S.st,     S.offers,      S.offT,   S.slab,
             S.L.slab_cap, S.pbest, 0,          S.btot,    S.in_mst};
  const int cus = S.cus;
  for (int mode : {kModeDense, kModeLds, kModeBucket, kModeGlobal}) {
    if (!(launched & (1 << mode))) continue;
    int grid;
    size_t lds;
    if (mode == kModeLds || mode == kModeDense) {
      lds = (size_t)scan_table_lds(mode, bound, S.dense_limit);
      // rounds >= 2: room for the round's label map (dom entries, 2 bytes
      // each, 1 in DENSE mode) behind the table, up to the LDS a workgroup
      // may take; the kernel lays out the table for the actual count and
      // stages as much of the map as then fits
      if (stage >= 2 && dom > 0)
        lds = std::min<size_t>((size_t)kMaxDynLds,
                               ((lds + 15) & ~size_t(15)) + (mode == kModeDense ? 1 : 2) * (size_t)dom);
      if (mode == kModeDense) {
        grid = std::min(S.L.nseg, cus);
      } else {
        const int occ = g_scan_occupancy.load();
        const int64_t fit = (int64_t)(160 * 1024) / ((int64_t)lds + 1024);  // LDS of one CU
        const int per_cu = (int)std::max<int64_t>(
            1, occ > 0 ? std::min<int64_t>(occ, fit) : std::min<int64_t>(4, 65536 / ((int64_t)lds + 1024)));
        grid = std::min(S.L.nseg, cus * per_cu);
      }
    } else if (mode == kModeBucket) {
      lds = kBucketScanLds;
      grid = std::min(S.L.nseg, cus);
    } else {
      lds = 0;
      grid = std::min(S.L.nseg, 2 * cus);
    }
    A.lds_bytes = (int32_t)lds;
    const int k = T.start(scan_kind(stage, mode), r, mode);
    err = launch_scan(mode, stage, A, grid, lds, S.s);
    T.stop(k);
    if (err != hipSuccess) return launched;
    if ((mode == kModeLds || mode == kModeDense) && S.slab) {
      const int ks = T.start(kSlabMin_, r, mode);
      const int64_t cols =
          mode == kModeDense ? kDensePairsMax : std::min<int64_t>(std::max<int64_t>(bound, 1), kLdsSlots);
      err = launch_slab_min(r, launched, mode, S.slab, S.L.slab_cap, grid, S.best, S.pbest, S.st, grid_for(cols),
                            S.s);
      T.stop(ks);
      if (err != hipSuccess) return launched;
    }
    if (mode == kModeDense && S.in_mst) {
      const int kd = T.start(kDenseFinish, r, mode);
      err = launch_dense_finish(r, launched, S.pbest, S.seg_live, S.L.nseg, S.rec, S.in_mst, S.total, S.st,
                                S.rounds, S.s);
      T.stop(kd);
      if (err != hipSuccess) return launched;
    }
    if (mode == kModeBucket) {
      const BucketGeom bg = bucket_geometry((int32_t)std::min<int64_t>(bound, kBucketMaxComponents));
      const int nbk = bg.nbk;
      // a smaller actual count can have more (narrower) buckets, but never more than 256
      // unless the width is at its maximum; the extra workgroups serve buckets with
      // more than twice the average offers (at most half as many again)
      const int grid_b = std::max(nbk, 256) * 3 / 2 + 1;
      const int kb = T.start(kBucketMin, r, kModeBucket);
      err = launch_bucket_min(r, launched, S.offers, S.offT, S.L.nseg, S.btot, S.best, S.st, grid_b,
                              (size_t)8 * bg.width, S.s);
      T.stop(kb);
      if (err != hipSuccess) return launched;
    }
  }
  return launched;
}

// Enqueues round r (component count at most `bound`; `exact`: the count is
// known to be `bound`, so only its own minima mode is launched).
// n_prev is the exact count entering round r - 1, which fixes the stream
// round r reads; its label map has n_prev entries, or, if round r - 1 kept
// its records untouched (S.keep[r - 1], known from round r - 2's record), as
// many as round r - 1's.
hipError_t enqueue_round(Solve& S, int r, int64_t bound, int64_t n_prev, bool exact) {
  LaunchTimer& T = t_timer;
  hipError_t err = hipSuccess;
  const int stage = scan_stage(r, n_prev);
  S.stage[r] = stage;
  S.dom[r] = r == 0 ? 0 : (S.keep[r - 1] == kKeepRecords ? S.dom[r - 1] : n_prev);
  S.launched[r] = enqueue_scan(S, r, stage, bound, exact, err, S.dom[r]);
  if (err != hipSuccess) return err;
  // the live edges two rounds before (the input's before round 1) are known
  // to every round loop when it enqueues round r, so every loop tries the
  // same rounds (the kernels check the exact count and mode themselves)
  const int64_t live_before = r >= 2 ? S.live_rec[r - 2] : S.m;
  if (r >= 1 && bound <= kSparseMaxK && S.sparse_limit > 0 && live_before <= S.sparse_limit &&
      (S.launched[r] & (1 << kModeLds))) {
    // few live edges left: try to end the solve on the graph of component pairs
    S.sparse_tried[r] = true;
    int k = T.start(kPairCollect, r, -1);
    err = launch_pair_collect(r, S.launched[r], S.rec, S.labpool, S.seg_cnt, S.L.nseg, S.sp, S.st,
                              std::min(S.L.nseg, 4 * S.cus), S.s);
    T.stop(k);
    if (err != hipSuccess) return err;
    k = T.start(kSparseFinish, r, -1);
    err = launch_sparse_finish(r, S.launched[r], S.rec, S.sp, S.seg_live, S.L.nseg, S.in_mst, S.total, S.st,
                               S.rounds, S.s);
    T.stop(k);
    if (err != hipSuccess) return err;
  }
  const int gh = grid_for(std::max<int64_t>(bound, 1));
  // a round that tried the sparse finish (bound <= kSparseMaxK <= kTailMax)
  // closes in one workgroup: one launch that returns when the finish ended
  // the solve, instead of four
  if (bound <= S.tail_limit || S.sparse_tried[r]) {
    // few components: the rest of the round in one workgroup
    const int k = T.start(kRoundTail, r, -1);
    err = launch_round_tail(r, (int32_t)bound, S.rec, S.best, S.parent, S.labpool, S.seg_cnt, S.seg_live,
                            S.L.nseg, S.in_mst, S.total, S.btot, S.st, S.rounds, S.s);
    T.stop(k);
    if (err != hipSuccess) return err;
    return S.events ? hipEventRecord(S.events[r], S.s) : hipSuccess;
  }
  int k = T.start(kHook, r, -1);
  err = launch_hook(r, S.rec, S.labpool, S.best, S.parent, S.st, S.in_mst, S.part_sel, S.part_w, gh, S.s);
  T.stop(k);
  if (err != hipSuccess) return err;
  k = T.start(kCompress, r, -1);
  err = launch_compress(r, S.parent, S.root_of, S.best, S.rootmask, S.rootcnt, S.st, gh, S.s);
  T.stop(k);
  if (err != hipSuccess) return err;
  k = T.start(kFinalize, r, -1);
  err = launch_finalize(r, S.rootcnt, S.rootpre, S.seg_cnt, S.seg_live, S.L.nseg, S.part_sel, S.part_w, gh,
                        S.st, S.total, S.rounds, S.s);
  T.stop(k);
  if (err != hipSuccess) return err;
  k = T.start(kRelabel, r, -1);
  err = launch_relabel(r, S.root_of, S.rootmask, S.rootpre, S.labpool, S.parent, S.best, S.btot, S.st, gh, S.s);
  T.stop(k);
  if (err != hipSuccess) return err;
  return S.events ? hipEventRecord(S.events[r], S.s) : hipSuccess;
}

// A round record as the device left it in pinned host memory (read through
// volatile accesses: the device writes it behind the compiler's back).
constexpr int32_t kRecordPending = -2;
HostRound load_record(const HostRound* p) {
  const volatile HostRound* v = p;
  HostRound h;
  h.n_next = v->n_next;
  h.err = v->err;
  h.err_internal = v->err_internal;
  h.dense = v->dense;
  h.live = v->live;
  h.sel = v->sel;
  h.edges_added = v->edges_added;
  h.stream = v->stream;
  h.map_n = v->map_n;
  h.keep = v->keep;
  h.keep_next = v->keep_next;
  std::atomic_thread_fence(std::memory_order_acquire);
  return h;
}

// The round loop of one graph (n >= 1, m >= 1) on a workspace of at least
// plan(n, m).bytes; the device cache is locked by the caller.
// The solve state of a graph on the workspace at B laid out by L; round
// records go to `rounds` (one per round), and `events` (if not null) are
// recorded after each round.
Solve make_solve(void* B, int cus, HostRound* rounds, hipEvent_t* events, const Layout& L, int32_t n, int64_t m,
                 const int32_t* src, const int32_t* dst, const uint32_t* w, uint8_t* in_mst, uint64_t* total,
                 hipStream_t s) {
  Solve S{};
  S.n = n;
  S.m = m;
  S.src = src;
  S.dst = dst;
  S.w = w;
  S.in_mst = in_mst;
  S.total = reinterpret_cast<unsigned long long*>(total);
  S.s = s;
  S.cus = cus;
  S.rounds = rounds;
  S.events = events;
  S.L = L;
  S.best = at<unsigned long long>(B, L.best);
  S.parent = at<int32_t>(B, L.parent);
  S.root_of = at<int32_t>(B, L.root_of);
  S.labpool = at<int32_t>(B, L.labpool);
  S.rootmask = at<unsigned long long>(B, L.rootmask);
  S.rootcnt = at<int32_t>(B, L.rootcnt);
  S.rootpre = at<int32_t>(B, L.rootpre);
  S.rec = at<uint4>(B, L.rec);
  S.seg_cnt = at<uint32_t>(B, L.seg_cnt);
  S.seg_live = at<uint32_t>(B, L.seg_live);
  S.part_sel = at<uint32_t>(B, L.part_sel);
  S.part_w = at<unsigned long long>(B, L.part_w);
  S.st = at<DevState>(B, L.state);
  S.offers = L.bucket ? at<unsigned long long>(B, L.offers) : nullptr;
  S.offT = L.bucket ? at<uint32_t>(B, L.offT) : nullptr;
  S.slab = L.slab_cap ? at<unsigned long long>(B, L.slab) : nullptr;
  S.pbest = at<unsigned long long>(B, L.pbest);
  S.btot = at<uint32_t>(B, L.btot);
  S.sp = SparseTable{at<uint32_t>(B, L.sp_pid), at<unsigned long long>(B, L.sp_key), at<uint32_t>(B, L.sp_state)};
  S.dense_limit = g_dense_limit.load();
  S.sparse_limit = g_sparse_limit.load();
  for (int64_t& x : S.live_rec) x = m;
  for (bool& x : S.sparse_tried) x = false;
  S.tail_limit = g_tail_limit.load();
  S.bucket_limit = g_bucket_limit.load();
  for (int& x : S.launched) x = 0;
  for (int& x : S.keep) x = 0;
  return S;
}

// Algorithmic bytes of round r's scan: the edge stream read once (12 B per
// input edge, 16 B per wide record, 8 B per narrow record, plus its 4-byte
// edge index when the round compacts it), the round's label map read once
// (4 B per entry), the minima initialised and written once (16 B per
// component), the survivors written once (16 B wide, 12 B narrow with the
// edge index; none when the round keeps its records, every record's 8 B when
// it relabels them in place); a dense round instead writes its pair table
// once (8 B per pair) and moves no record.
double round_scan_bytes(const HostRound* rec, const int32_t* nr_of, int r, int64_t m) {
  const HostRound& M = rec[r];
  const double nrd = (double)nr_of[r];
  const bool narrow_in = r >= 2 && nr_of[r - 1] <= kNarrowMax;
  const bool dense = M.dense == 1;  // the dense finish's round (2: the sparse finish, an LDS round)
  const bool moves = r >= 1 && !dense && M.keep == kMoveRecords;
  const bool relabels = !dense && M.keep == kRelabelRecords;
  double b = r <= 1 ? 12.0 * (double)m : (narrow_in ? (moves ? 12.0 : 8.0) : 16.0) * (double)M.stream;
  b += 4.0 * (double)M.map_n;
  b += dense ? 8.0 * (double)dense_pairs(nr_of[r]) : 16.0 * nrd;
  if (moves) b += (nr_of[r] <= kNarrowMax ? 12.0 : 16.0) * (double)M.live;
  if (relabels) b += 8.0 * (double)M.stream;
  return b;
}

// Algorithmic bytes of round r's kernels other than the scan and the bucket
// minima (all bound by latency: random gathers, one-workgroup chains), per
// component c of the n_r: the hook reads best[c], the record at its key (the
// 4-byte end xor in round 0, a 12-byte narrow record with its edge index,
// else 16 B) and best of the far end, and writes parent and in_mst of the
// s_r components that hook; compress reads a parent and best[c] and writes
// the root (16 B, bits aside); finalize reads and writes one word per 64
// components and two counts per segment; relabel reads the root, its mask
// word and prefix and writes the label (20 B), and resets the next round's
// minimum and parent (12 B per component of round r + 1); the round tail
// does hook, relabel and resets in one (best, record, label, in_mst, resets);
// the dense finish reads its pair table once.  Walks longer than one step
// and the composed label maps are not counted.
void other_bytes(const HostRound* rec, const int32_t* nr_of, int r, int nseg, bool sparse_tried,
                 double (&out)[kKinds]) {
  for (double& x : out) x = 0.0;
  const HostRound& M = rec[r];
  const double n = (double)nr_of[r], nn = (double)M.n_next, sel = (double)M.sel;
  const double recb = r == 0 ? 4.0 : (nr_of[r] <= kNarrowMax ? 12.0 : 16.0);
  if (sparse_tried) {
    // the pair collection reads every live record once (8 B) and lowers a
    // 12-byte pair slot for it; the finish reads and empties the table
    out[kPairCollect] = 20.0 * (double)M.live;
    out[kSparseFinish] = 24.0 * (double)kSparseHash + 8.0 * (double)nseg;
  }
  if (M.dense == 1) {
    out[kDenseFinish] = 8.0 * (double)dense_pairs(nr_of[r]);
    return;
  }
  if (M.dense == 2) return;  // the sparse finish ended the solve: no hook or relabel ran
  out[kHook] = (16.0 + recb) * n + 5.0 * sel;
  out[kCompress] = 16.0 * n;
  out[kFinalize] = 8.0 * n / 64.0 + 8.0 * (double)nseg;
  out[kRelabel] = 20.0 * n + 12.0 * nn;
  out[kRoundTail] = (8.0 + recb + 4.0) * n + 5.0 * sel + 12.0 * nn + 8.0 * (double)nseg;
}

// What the host learns from the round records of one solve.
struct RoundLoop {
  int32_t n = 0;
  int rounds = 0;                 // records taken
  int status = MSTX_ERR_DEVICE;   // until a record decides
  bool done = false;
  int32_t nr_of[kMaxRounds + 2];  // exact component count entering round r (r <= rounds)

  explicit RoundLoop(int32_t n0) : n(n0) {
    for (int32_t& x : nr_of) x = 0;
    nr_of[0] = n0;
  }
  // Takes round r's record (r == rounds); sets `done` when the solve ends.
  void take(int r, const HostRound& M) {
    rounds = r + 1;
    if (r == 0 && M.err) {
      status = MSTX_ERR_VERTEX_RANGE;
      done = true;
    } else if (M.err_internal) {
      status = MSTX_ERR_DEVICE;
      done = true;
    } else {
      nr_of[r + 1] = M.n_next;
      if (M.n_next <= 1) {
        status = (n <= 1 || M.edges_added == (int64_t)n - 1) ? MSTX_OK : MSTX_DISCONNECTED;
        done = true;
      }
    }
  }
  // Statistics of the finished solve for mst_last_round_stats, and the
  // profile's per-round modes and bytes.
  void finish(const Solve& S, const HostRound* rec, int64_t m) const {
    RoundStats& T = t_last_stats;
    T.rounds = rounds;
    int chosen[kMaxRounds + 1];
    double bytes[kMaxRounds + 1], bmin[kMaxRounds + 1];
    double other[kMaxRounds + 1][kKinds];
    for (int r = 0; r < rounds; ++r) {
      other_bytes(rec, nr_of, r, S.L.nseg, S.sparse_tried[r], other[r]);
      T.v[3 * r + 0] = nr_of[r];
      T.v[3 * r + 1] = rec[r].live;
      T.v[3 * r + 2] = rec[r].sel;
      chosen[r] = pick_mode(nr_of[r], S.launched[r]);
      bytes[r] = round_scan_bytes(rec, nr_of, r, m);
      // bucket minima: two 8-byte offers per live edge read, one 8-byte minimum per component written
      bmin[r] = 16.0 * (double)rec[r].live + 8.0 * (double)nr_of[r];
    }
    t_timer.commit(rounds, chosen, bytes, bmin, other);
  }
};

// S0 of a solve on the stream: outputs zeroed, minima, parents and state reset.
hipError_t start_solve(const Solve& S) {
  hipError_t e = hipMemsetAsync(S.in_mst, 0, (size_t)S.m, S.s);
  if (e == hipSuccess) e = hipMemsetAsync(S.total, 0, sizeof(uint64_t), S.s);
  if (e == hipSuccess)
    e = launch_init(S.n, S.m, (int64_t)((S.L.cmap - S.L.labpool) / 4), S.dense_limit, S.best, S.parent,
                    S.dense_limit > 0 ? S.pbest : nullptr, S.btot, S.sp, S.st, grid_for(S.n), S.s);
  return e;
}

// The rounds of one solve as a state machine.  start() enqueues S0 and
// round 0; advance() takes every round record that has arrived and enqueues
// the next round as the pipelining allows (round r + 1 is enqueued before
// round r's record is waited for); with `block` it waits for each record,
// otherwise it returns at the first record not there yet.  When the solve
// has ended it drains the stream and publishes the round statistics.
struct RoundMachine {
  Solve S;
  RoundLoop R;
  HostRound* rec;
  hipEvent_t* ev;
  int64_t m;
  int max_rounds;
  int r = 0;            // next round whose record is taken
  int r_enq = 0;        // last round enqueued
  int32_t n_known = 0;  // exact component count entering round r
  bool done = false;

  RoundMachine(void* base, int cus, HostRound* rec_, hipEvent_t* ev_, const Layout& L, int32_t n, int64_t m_,
               const int32_t* src, const int32_t* dst, const uint32_t* w, uint8_t* in_mst, uint64_t* total,
               hipStream_t s)
      : S(make_solve(base, cus, rec_, ev_, L, n, m_, src, dst, w, in_mst, total, s)),
        R(n),
        rec(rec_),
        ev(ev_),
        m(m_),
        max_rounds(std::min(rounds_bound(n) + 1, kMaxRounds)),
        n_known(n) {}

  int start() {
    HIP_OK(start_solve(S));
    // every record reads "pending" until the device writes it
    for (int q = 0; q <= kMaxRounds; ++q) rec[q].n_next = kRecordPending;
    std::atomic_thread_fence(std::memory_order_seq_cst);
    HIP_OK(enqueue_round(S, 0, S.n, 0, true));
    return MSTX_OK;
  }

  // one_round: return once a record has been taken and the rounds after it
  // are enqueued as far as the pipelining allows (a blocking call then waits
  // for one round only)
  int advance(bool block, bool one_round = false) {
    bool took = false;
    while (!done) {
      if (r >= max_rounds) {
        done = true;  // round-count watchdog: status stays MSTX_ERR_DEVICE
        break;
      }
      if (r_enq < r) {
        // round r - 1 tried the sparse finish and went on: round r was not
        // enqueued ahead, and its count is known exactly now
        HIP_OK(enqueue_round(S, r, n_known, R.nr_of[r - 1], true));
        r_enq = r;
      }
      // a round whose scan takes the dense finish (its count n_known is exact
      // here) is the last one: nothing to enqueue after it; a round that tries
      // the sparse finish usually is, so the next one waits for its record
      const bool final_round = pick_mode(n_known, S.launched[r]) == kModeDense;
      if (r_enq == r && r + 1 <= kMaxRounds - 1 && !final_round && !S.sparse_tried[r]) {
        // n_known entered round r: the size of the label map round r + 1 reads
        HIP_OK(enqueue_round(S, r + 1, n_known / 2, n_known, false));
        r_enq = r + 1;
      }
      if (one_round && took) return MSTX_OK;
      if (block) {
        HIP_OK(hipEventSynchronize(ev[r]));
      } else {
        const hipError_t q = hipEventQuery(ev[r]);
        if (q == hipErrorNotReady) {
          (void)hipGetLastError();
          return MSTX_OK;
        }
        HIP_OK(q);
      }
      HostRound M = load_record(rec + r);
      if (M.n_next == kRecordPending) {
        // not visible yet: wait for the whole stream, then it must be
        HIP_OK(hipStreamSynchronize(S.s));
        M = load_record(rec + r);
        if (M.n_next == kRecordPending) {
          done = true;  // status stays MSTX_ERR_DEVICE
          break;
        }
      }
      R.take(r, M);
      took = true;
      S.keep[r + 1] = M.keep_next;
      S.live_rec[r] = M.live;
      if (R.done) {
        done = true;
        break;
      }
      n_known = M.n_next;
      ++r;
    }
    HIP_OK(hipStreamSynchronize(S.s));  // drains the round enqueued after the last one
    if (R.status >= 0) R.finish(S, rec, m);
    return MSTX_OK;
  }
};

int solve_locked(DeviceCache* dc, const Layout& L, int32_t n, int64_t m, const int32_t* src, const int32_t* dst,
                 const uint32_t* w, uint8_t* in_mst, uint64_t* total, hipStream_t s) {
  RoundMachine M(dc->base, dc->cus, dc->host_rounds, dc->round_ev, L, n, m, src, dst, w, in_mst, total, s);
  t_timer.begin(s);
  int rc = M.start();
  if (rc != MSTX_OK) return rc;
  rc = M.advance(true);
  if (rc != MSTX_OK) return rc;
  return M.R.status;
}

// A graph of at most kSmallN vertices in one launch (the batched path's
// one-workgroup solve); the cache is locked by the caller.
int solve_small_locked(DeviceCache* dc, int32_t n, int64_t m, const int32_t* src, const int32_t* dst,
                       const uint32_t* w, uint8_t* in_mst, uint64_t* total, hipStream_t s) {
  const size_t words = 1 + kSmallStatsWords;  // status word, then the statistics
  if (!dc->small_dev) {
    if (hipMalloc(&dc->small_dev, 8 * words) != hipSuccess) {
      (void)hipGetLastError();
      dc->small_dev = nullptr;
      return MSTX_ERR_OUT_OF_MEMORY;
    }
    HIP_OK(hipHostMalloc((void**)&dc->small_host, 8 * words, hipHostMallocDefault));
  }
  int64_t* dev = static_cast<int64_t*>(dc->small_dev);
  LaunchTimer& T = t_timer;
  T.begin(s);
  HIP_OK(hipMemsetAsync(in_mst, 0, (size_t)m, s));
  const int k = T.start(kSmallSolve, 0, -1);
  HIP_OK(launch_small_solve_single(n, m, src, dst, w, in_mst, reinterpret_cast<unsigned long long*>(total),
                                   reinterpret_cast<int32_t*>(dev), dev + 1, s));
  T.stop(k);
  HIP_OK(hipMemcpyAsync(dc->small_host, dev, 8 * words, hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  const int32_t status = *reinterpret_cast<const int32_t*>(dc->small_host);
  const int64_t* st = dc->small_host + 1;
  const int rows = (int)std::min<int64_t>(std::max<int64_t>(st[0], 0), kMaxRounds + 1);
  // algorithmic bytes: every round reads the 12-byte edges once, plus one
  // final round that finds nothing to add
  T.commit(0, nullptr, nullptr, nullptr, nullptr);
  if (T.on) {
    std::lock_guard<std::mutex> g(g_prof.mu);
    g_prof.bytes[kSmallSolve] += 12.0 * (double)m * (double)(rows + 1);
  }
  if (status < 0) return status;
  t_last_stats.rounds = rows;
  std::memcpy(t_last_stats.v, st + 1, sizeof(int64_t) * 3 * (size_t)rows);
  return status;
}

int solve(int32_t n, int64_t m, const int32_t* src, const int32_t* dst, const uint32_t* w, uint8_t* in_mst,
          uint64_t* total, hipStream_t s) {
  t_last_stats.clear();
  const Layout L = plan(n, m);
  if (L.bytes > workspace_limit()) return MSTX_ERR_OUT_OF_MEMORY;
  if (m == 0) {
    HIP_OK(hipMemsetAsync(total, 0, sizeof(uint64_t), s));
    HIP_OK(hipStreamSynchronize(s));
    return n <= 1 ? MSTX_OK : MSTX_DISCONNECTED;
  }
  if (n == 0) return MSTX_ERR_VERTEX_RANGE;  // m > 0 edges, no valid vertex id
  DeviceCache* dc = nullptr;
  std::unique_lock<std::mutex> lock;
  if (n <= g_small_limit.load() && m <= kSmallMaxEdges) {
    // one workgroup runs every round with the vertex state in LDS
    int rc = acquire(dc, lock, 0, s);
    if (rc != MSTX_OK) return rc;
    return solve_small_locked(dc, n, m, src, dst, w, in_mst, total, s);
  }
  int rc = acquire(dc, lock, L.bytes, s);
  if (rc != MSTX_OK) return rc;
  return solve_locked(dc, L, n, m, src, dst, w, in_mst, total, s);
}

// ------------------------------------------------------ allocation-free solve

// One device's state of mst_solve_noalloc: the device address of its copy of
// `scratch` and a lock that serialises the calls on that device (they share
// the scratch; each call has finished its device work when it returns, so
// calls never overlap on it).
struct NoAllocDevice {
  std::mutex mu;
  unsigned char* ptr = nullptr;
  int cus = 0;
};
constexpr int kNoAllocDevices = 64;
NoAllocDevice g_noalloc[kNoAllocDevices];
constexpr size_t kNoAllocRecordBytes = align_up(sizeof(HostRound) * (kMaxRounds + 1));

// First call on the current device `dev`: the scratch's device address and
// the kernels' LDS limits.  No allocation.
int noalloc_setup(NoAllocDevice& D, int dev) {
  if (D.ptr) return MSTX_OK;
  void* p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) {
    (void)hipGetLastError();
    return MSTX_ERR_DEVICE;
  }
  int cus = 0;
  HIP_OK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  if (configure_kernels() != hipSuccess) (void)hipGetLastError();
  if (configure_batched_kernels() != hipSuccess) (void)hipGetLastError();
  D.cus = cus;
  D.ptr = static_cast<unsigned char*>(p);
  return MSTX_OK;
}

// solve() without allocating: the same kernels on this device's scratch.  The
// round records are written to device memory and copied into the host's
// stack after each synchronisation (no pinned memory, no events); each
// synchronisation covers two rounds: the next one at its exact component
// count and the one after it at the bound of half that count.
int solve_noalloc(int32_t n, int64_t m, const int32_t* src, const int32_t* dst, const uint32_t* w, uint8_t* in_mst,
                  uint64_t* total, hipStream_t s) {
  t_last_stats.clear();
  if (m == 0) {
    HIP_OK(hipMemsetAsync(total, 0, sizeof(uint64_t), s));
    HIP_OK(hipStreamSynchronize(s));
    return n <= 1 ? MSTX_OK : MSTX_DISCONNECTED;
  }
  if (n == 0) return MSTX_ERR_VERTEX_RANGE;
  const bool small = n <= g_small_limit.load() && m <= kSmallMaxEdges;
  const Layout L = plan(n, m);
  if (!small && L.bytes + kNoAllocRecordBytes > kNoAllocScratchBytes) return MSTX_ERR_SCRATCH_LIMIT;
  int dev = 0;
  HIP_OK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kNoAllocDevices) return MSTX_ERR_DEVICE;
  NoAllocDevice& D = g_noalloc[dev];
  std::lock_guard<std::mutex> lock(D.mu);
  int rc = noalloc_setup(D, dev);
  if (rc != MSTX_OK) return rc;
  t_timer.begin(s);
  t_timer.on = false;  // profiling events are not created here

  if (small) {
    // status word, then the statistics, at the start of the scratch
    int64_t* words = reinterpret_cast<int64_t*>(D.ptr);
    int64_t host[1 + kSmallStatsWords];
    HIP_OK(hipMemsetAsync(in_mst, 0, (size_t)m, s));
    HIP_OK(launch_small_solve_single(n, m, src, dst, w, in_mst, reinterpret_cast<unsigned long long*>(total),
                                     reinterpret_cast<int32_t*>(words), words + 1, s));
    HIP_OK(hipMemcpyAsync(host, words, sizeof(host), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    const int32_t status = *reinterpret_cast<const int32_t*>(host);
    if (status < 0) return status;
    const int rows = (int)std::min<int64_t>(std::max<int64_t>(host[1], 0), kMaxRounds + 1);
    t_last_stats.rounds = rows;
    std::memcpy(t_last_stats.v, host + 2, sizeof(int64_t) * 3 * (size_t)rows);
    return status;
  }

  HostRound* drec = reinterpret_cast<HostRound*>(D.ptr + L.bytes);
  Solve S = make_solve(D.ptr, D.cus, drec, nullptr, L, n, m, src, dst, w, in_mst, total, s);
  const int max_rounds = std::min(rounds_bound(n) + 1, kMaxRounds);
  HIP_OK(start_solve(S));
  HIP_OK(hipMemsetAsync(drec, 0xFF, kNoAllocRecordBytes, s));  // n_next = -1 until written
  HIP_OK(enqueue_round(S, 0, n, 0, true));
  int r_enq = 0;
  if (pick_mode(n, S.launched[0]) != kModeDense && max_rounds > 1) {
    HIP_OK(enqueue_round(S, 1, n / 2, n, false));
    r_enq = 1;
  }
  RoundLoop R(n);
  HostRound h[kMaxRounds + 1];
  for (;;) {
    HIP_OK(hipMemcpyAsync(h, drec, sizeof(h), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    // every enqueued round has finished: its record is there
    for (int r = R.rounds; r <= r_enq && !R.done; ++r) {
      if (h[r].n_next < 0) {
        R.done = true;  // never: a finished round wrote its record
        break;
      }
      R.take(r, h[r]);
      S.keep[r + 1] = h[r].keep_next;
      S.live_rec[r] = h[r].live;
    }
    if (R.done) break;
    const int r = r_enq + 1;  // its component count is known exactly now
    if (r >= max_rounds) break;  // round-count watchdog: MSTX_ERR_DEVICE
    const int32_t nk = R.nr_of[r];
    HIP_OK(enqueue_round(S, r, nk, R.nr_of[r - 1], true));
    r_enq = r;
    if (pick_mode(nk, S.launched[r]) != kModeDense && r + 1 < max_rounds) {
      HIP_OK(enqueue_round(S, r + 1, nk / 2, nk, false));
      r_enq = r + 1;
    }
  }
  if (R.status < 0) return R.status;
  R.finish(S, h, m);
  return R.status;
}

// ---------------------------------------------------------- stepwise solve

// A solve advanced round by round by the caller (mst_solve_begin ..
// mst_solve_end), on the stepwise workspace of its (device, stream): at most
// one per stream at a time.  Other calls on the stream run between its rounds.
struct StepSolve {
  DeviceCache* dc = nullptr;
  std::unique_ptr<RoundMachine> rm;
  hipStream_t s = nullptr;
  int status = MSTX_ERR_DEVICE;
  bool done = false;
};

void step_release(StepSolve* h) {
  if (!h->dc) return;
  std::lock_guard<std::mutex> g(h->dc->mu);
  h->dc->step_active = false;
  h->dc = nullptr;
}

int step_begin(int32_t n, int64_t m, const int32_t* src, const int32_t* dst, const uint32_t* w, uint8_t* in_mst,
               uint64_t* total, hipStream_t s, StepSolve** out) {
  *out = nullptr;
  t_last_stats.clear();
  std::unique_ptr<StepSolve> h(new StepSolve());
  h->s = s;
  const Layout L = plan(n, m);
  if (m == 0 || (n > 0 && n <= g_small_limit.load() && m <= kSmallMaxEdges)) {
    // nothing to step: no edges, or one launch of the one-workgroup solve
    const int st = solve(n, m, src, dst, w, in_mst, total, s);
    if (st < 0) return st;
    h->status = st;
    h->done = true;
    *out = h.release();
    return MSTX_OK;
  }
  if (n == 0) return MSTX_ERR_VERTEX_RANGE;
  if (L.bytes > workspace_limit()) return MSTX_ERR_OUT_OF_MEMORY;
  DeviceCache* dc = nullptr;
  {
    std::unique_lock<std::mutex> lock;
    int rc = acquire(dc, lock, 0, s);
    if (rc != MSTX_OK) return rc;
    if (dc->step_active) return MSTX_ERR_INVALID_ARG;  // one stepwise solve per stream
    if (!dc->step_rounds) {
      HIP_OK(hipHostMalloc((void**)&dc->step_rounds, sizeof(HostRound) * (kMaxRounds + 1), hipHostMallocDefault));
      for (int i = 0; i <= kMaxRounds; ++i)
        HIP_OK(hipEventCreateWithFlags(&dc->step_ev[i], hipEventDisableTiming | hipEventDisableSystemFence));
    }
    if (dc->step_bytes < L.bytes) {
      if (dc->step_base) {
        HIP_OK(hipFreeAsync(dc->step_base, s));
        dc->step_base = nullptr;
        dc->step_bytes = 0;
      }
      if (hipMallocAsync(&dc->step_base, L.bytes, s) != hipSuccess) {
        (void)hipGetLastError();
        dc->step_base = nullptr;
        return MSTX_ERR_OUT_OF_MEMORY;
      }
      dc->step_bytes = L.bytes;
    }
    dc->step_active = true;
  }
  h->dc = dc;
  h->rm.reset(new RoundMachine(dc->step_base, dc->cus, dc->step_rounds, dc->step_ev, L, n, m, src, dst, w, in_mst,
                               total, s));
  t_timer.begin(s);
  t_timer.on = false;  // per-launch timing covers blocking solves only
  const int rc = h->rm->start();
  if (rc != MSTX_OK) {
    step_release(h.get());
    return rc;
  }
  *out = h.release();
  return MSTX_OK;
}

int step_advance(StepSolve* h, bool block, bool one_round = false) {
  if (h->done) return MSTX_OK;
  t_timer.begin(h->s);
  t_timer.on = false;
  const int rc = h->rm->advance(block, one_round);
  if (rc != MSTX_OK || h->rm->done) {
    h->done = true;
    h->status = rc != MSTX_OK ? rc : h->rm->R.status;
    step_release(h);
  }
  return MSTX_OK;
}

// ----------------------------------------------------------------- batched

// Which path a graph of a batch takes: one workgroup with everything in LDS
// (small); one workgroup with the edges streamed every round (mid); one
// workgroup contracting it round by round until at most mid_limit components
// are left, then the mid path on those (contract); or every round in a chunk
// of the disjoint union solved by the round kernels (large).
// A graph with more than kMidMaxEdges edges goes to the union whatever its
// vertex count: one workgroup would stream all of them every round.
enum class BatchPath { kSmall, kMid, kContract, kLarge };
BatchPath batch_path(int64_t n, int64_t m, int32_t mid_limit) {
  if (m > kMidMaxEdges) return BatchPath::kLarge;
  // the small solve when its LDS also holds the edges (or the mid-size path
  // is off); otherwise the mid-size solve, whose dense finish saves passes
  if (n <= kSmallN && (small_edges_cached(n, m) || mid_limit <= kSmallN)) return BatchPath::kSmall;
  if (mid_limit > kSmallN) {
    if (n <= mid_limit) return BatchPath::kMid;
    if (n <= kPreMaxN) return BatchPath::kContract;
  }
  return BatchPath::kLarge;
}

// Device scratch of a batched call besides the solve workspace.
struct BatchLayout {
  size_t voff, eoff, small, mid, large, cvert, cedge, gbad, gsrc, gdst, gw, cin, total, acc_w, acc_c, con, cpoff,
      csoff, cscratch, cnum, pcnt, pbad, pairs, bytes;
};

// ncon graphs are contracted, with con_n vertices and con_m edges in all.
BatchLayout plan_batch(int32_t G, int64_t nsmall, int64_t nmid, int64_t nlarge, int64_t nchunk_meta,
                       int64_t max_chunk_m, int64_t ncon, int64_t con_n, int64_t con_m) {
  BatchLayout B{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  B.voff = take(8 * ((size_t)G + 1));
  B.eoff = take(8 * ((size_t)G + 1));
  B.small = take(4 * (size_t)std::max<int64_t>(nsmall, 1));
  B.mid = take(4 * (size_t)std::max<int64_t>(nmid, 1));
  B.large = take(4 * (size_t)std::max<int64_t>(nlarge, 1));
  B.cvert = take(8 * (size_t)std::max<int64_t>(nchunk_meta, 1));
  B.cedge = take(8 * (size_t)std::max<int64_t>(nchunk_meta, 1));
  B.gbad = take(4 * (size_t)std::max<int64_t>(nlarge, 1));
  B.gsrc = take(4 * (size_t)std::max<int64_t>(max_chunk_m, 1));
  B.gdst = take(4 * (size_t)std::max<int64_t>(max_chunk_m, 1));
  B.gw = take(4 * (size_t)std::max<int64_t>(max_chunk_m, 1));
  B.cin = take((size_t)std::max<int64_t>(max_chunk_m, 1));
  B.total = take(8);
  B.acc_w = take(8 * (size_t)std::max<int64_t>(nlarge, 1));
  B.acc_c = take(4 * (size_t)std::max<int64_t>(nlarge, 1));
  B.con = take(4 * (size_t)std::max<int64_t>(ncon, 1));
  B.cpoff = take(8 * (size_t)std::max<int64_t>(ncon, 1));
  B.csoff = take(8 * (size_t)std::max<int64_t>(ncon, 1));
  B.cscratch = take(8 * (size_t)std::max<int64_t>(con_n, 1));
  B.cnum = take(4 * (size_t)std::max<int64_t>(ncon, 1));
  B.pcnt = take(4 * (size_t)std::max<int64_t>(ncon, 1));
  B.pbad = take(4 * (size_t)std::max<int64_t>(ncon, 1));
  B.pairs = take(4 * (size_t)std::max<int64_t>(con_m, 1));
  B.bytes = off;
  return B;
}

int grow_aux(DeviceCache* dc, size_t bytes, hipStream_t stream) {
  if (dc->aux_bytes >= bytes) return MSTX_OK;
  // stream-ordered, as the workspace in acquire()
  if (dc->aux) {
    HIP_OK(hipFreeAsync(dc->aux, stream));
    dc->aux = nullptr;
    dc->aux_bytes = 0;
  }
  if (hipMallocAsync(&dc->aux, bytes, stream) != hipSuccess) {
    (void)hipGetLastError();
    dc->aux = nullptr;
    return MSTX_ERR_OUT_OF_MEMORY;
  }
  dc->aux_bytes = bytes;
  return MSTX_OK;
}

int check_batch_args(int32_t G, const int64_t* voff, const int64_t* eoff, const void* src, const void* dst,
                     const void* w, const void* in_mst, const void* total, const void* status) {
  if (G < 0) return MSTX_ERR_INVALID_ARG;
  if (G == 0) return MSTX_OK;
  if (!voff || !eoff || !total || !status) return MSTX_ERR_INVALID_ARG;
  if (voff[0] != 0 || eoff[0] != 0) return MSTX_ERR_INVALID_ARG;
  for (int32_t g = 0; g < G; ++g) {
    if (voff[g + 1] < voff[g] || eoff[g + 1] < eoff[g]) return MSTX_ERR_INVALID_ARG;
    if (voff[g + 1] - voff[g] > (int64_t)INT32_MAX) return MSTX_ERR_INVALID_ARG;
    if (eoff[g + 1] - eoff[g] > (int64_t)0xFFFFFFFFLL) return MSTX_ERR_TOO_LARGE;
  }
  if (eoff[G] > 0 && (!src || !dst || !w || !in_mst)) return MSTX_ERR_INVALID_ARG;
  return MSTX_OK;
}

// How a batch is split: the graphs of each path and the union chunks.
struct BatchPlan {
  std::vector<int32_t> small, mid, con, uni;
  // chunk c: uni[cfirst[c] .. cfirst[c + 1]); its graphs' vertex and edge
  // offsets inside the union are cvert / cedge[meta_at[c] ..] (ng + 1 each)
  std::vector<int32_t> cfirst;
  std::vector<int64_t> cvert, cedge, meta_at;
  std::vector<int64_t> cpoff, csoff;  // contracted graph i: start of its edge pairs, of its scratch
  int64_t con_n = 0, con_m = 0;
  int64_t max_chunk_n = 0, max_chunk_m = 0;
  int32_t mid_max_n = 0;
};

BatchPlan plan_batch_graphs(int32_t G, const int64_t* voff, const int64_t* eoff, int32_t mid_limit) {
  BatchPlan P;
  for (int32_t g = 0; g < G; ++g) {
    switch (batch_path(voff[g + 1] - voff[g], eoff[g + 1] - eoff[g], mid_limit)) {
      case BatchPath::kSmall: P.small.push_back(g); break;
      case BatchPath::kMid: P.mid.push_back(g); break;
      case BatchPath::kContract: P.con.push_back(g); break;
      case BatchPath::kLarge: P.uni.push_back(g); break;
    }
  }
  // most edges first, so the longest workgroups of a launch start first
  auto more_edges = [&](int32_t a, int32_t b) { return eoff[a + 1] - eoff[a] > eoff[b + 1] - eoff[b]; };
  for (auto* v : {&P.small, &P.mid, &P.con, &P.uni}) std::stable_sort(v->begin(), v->end(), more_edges);
  for (int32_t g : P.mid) P.mid_max_n = std::max<int32_t>(P.mid_max_n, (int32_t)(voff[g + 1] - voff[g]));
  for (int32_t g : P.con) {
    P.cpoff.push_back(P.con_m);
    P.csoff.push_back(P.con_n);
    P.con_m += eoff[g + 1] - eoff[g];
    P.con_n += voff[g + 1] - voff[g];
  }
  // chunks: consecutive graphs, union within the bucket-mode limit
  int64_t cn = 0, cm = 0;
  for (int32_t i = 0; i < (int32_t)P.uni.size(); ++i) {
    const int32_t g = P.uni[i];
    const int64_t ng = voff[g + 1] - voff[g], mg = eoff[g + 1] - eoff[g];
    if (i == 0 || cn + ng > kBucketMaxComponents || cm + mg > (int64_t)0xFFFFFFFFLL) {
      P.cfirst.push_back(i);
      cn = cm = 0;
    }
    cn += ng;
    cm += mg;
    P.max_chunk_n = std::max(P.max_chunk_n, cn);
    P.max_chunk_m = std::max(P.max_chunk_m, cm);
  }
  P.cfirst.push_back((int32_t)P.uni.size());
  for (size_t c = 0; c + 1 < P.cfirst.size(); ++c) {
    P.meta_at.push_back((int64_t)P.cvert.size());
    int64_t a = 0, b = 0;
    for (int32_t i = P.cfirst[c]; i < P.cfirst[c + 1]; ++i) {
      P.cvert.push_back(a);
      P.cedge.push_back(b);
      a += voff[P.uni[i] + 1] - voff[P.uni[i]];
      b += eoff[P.uni[i] + 1] - eoff[P.uni[i]];
    }
    P.cvert.push_back(a);
    P.cedge.push_back(b);
  }
  return P;
}

BatchLayout plan_batch(int32_t G, const BatchPlan& P) {
  return plan_batch(G, (int64_t)P.small.size(), (int64_t)P.mid.size(), (int64_t)P.uni.size(), (int64_t)P.cvert.size(),
                    P.max_chunk_m, (int64_t)P.con.size(), P.con_n, P.con_m);
}

// Every graph of the batch that one workgroup solves, in one launch: the
// contracted ones (their first rounds, then the mid-size solve on the at most
// mid_limit components left), the mid-size ones, the small ones.  The class
// lists and offsets are at their places in A (laid out by BL).
hipError_t launch_one_workgroup_classes(const BatchPlan& P, const BatchLayout& BL, void* A, int32_t mid_limit,
                                        const int32_t* src, const int32_t* dst, const uint32_t* w, uint8_t* in_mst,
                                        uint64_t* total, int32_t* status, hipStream_t s) {
  auto* d_voff = at<int64_t>(A, BL.voff);
  auto* d_eoff = at<int64_t>(A, BL.eoff);
  auto* d_small = at<int32_t>(A, BL.small);
  auto* d_mid = at<int32_t>(A, BL.mid);
  auto* d_con = at<int32_t>(A, BL.con);
  auto* d_cpoff = at<int64_t>(A, BL.cpoff);
  auto* d_csoff = at<int64_t>(A, BL.csoff);
  auto* d_cnum = at<int32_t>(A, BL.cnum);
  auto* d_pcnt = at<int32_t>(A, BL.pcnt);
  auto* d_pbad = at<int32_t>(A, BL.pbad);
  auto* d_pairs = at<uint32_t>(A, BL.pairs);
  auto* tot = reinterpret_cast<unsigned long long*>(total);
  const int32_t max_n = std::min<int32_t>(mid_limit, kMidN);
  BatchSolveArgs B{};
  B.pre = PreArgs{d_con,   d_voff,  d_eoff, src,    dst,    w,      d_csoff, at<unsigned long long>(A, BL.cscratch),
                  d_pairs, d_cpoff, d_cnum, d_pcnt, d_pbad, in_mst, tot,     max_n};
  B.con = MidArgs{d_con,  d_voff, d_eoff, nullptr, nullptr, w,   d_pairs, d_cpoff,
                  d_cnum, d_pcnt, d_pbad, in_mst,  tot,     status, max_n};
  B.mid = MidArgs{d_mid,   d_voff,  d_eoff,  src,    dst, w,      nullptr, nullptr,
                  nullptr, nullptr, nullptr, in_mst, tot, status, P.mid_max_n};
  B.small = MidArgs{d_small, d_voff,  d_eoff,  src,    dst, w,      nullptr, nullptr,
                    nullptr, nullptr, nullptr, in_mst, tot, status, 0};
  B.ncon = (int32_t)P.con.size();
  B.nmid = (int32_t)P.mid.size();
  return launch_batch_solve(B, (int)P.small.size(), s);
}

int solve_batched(int32_t G, const int64_t* voff, const int64_t* eoff, const int32_t* src, const int32_t* dst,
                  const uint32_t* w, uint8_t* in_mst, uint64_t* total, int32_t* status, hipStream_t s) {
  t_last_stats.clear();
  if (G == 0) return MSTX_OK;
  const int32_t mid_limit = g_mid_limit.load();
  const BatchPlan P = plan_batch_graphs(G, voff, eoff, mid_limit);
  if (P.max_chunk_n > INT32_MAX) return MSTX_ERR_TOO_LARGE;
  const int64_t nuni = (int64_t)P.uni.size(), ncon = (int64_t)P.con.size();
  const Layout L = plan((int32_t)std::max<int64_t>(P.max_chunk_n, 1), std::max<int64_t>(P.max_chunk_m, 1));
  const BatchLayout BL = plan_batch(G, P);
  if (L.bytes + BL.bytes > workspace_limit()) return MSTX_ERR_OUT_OF_MEMORY;

  DeviceCache* dc = nullptr;
  std::unique_lock<std::mutex> lock;
  int rc = acquire(dc, lock, nuni == 0 ? 0 : L.bytes, s);
  if (rc != MSTX_OK) return rc;
  rc = grow_aux(dc, BL.bytes, s);
  if (rc != MSTX_OK) return rc;
  void* A = dc->aux;
  auto* d_voff = at<int64_t>(A, BL.voff);
  auto* d_eoff = at<int64_t>(A, BL.eoff);
  auto* d_small = at<int32_t>(A, BL.small);
  auto* d_mid = at<int32_t>(A, BL.mid);
  auto* d_uni = at<int32_t>(A, BL.large);
  auto* d_cvert = at<int64_t>(A, BL.cvert);
  auto* d_cedge = at<int64_t>(A, BL.cedge);
  auto* d_gbad = at<int32_t>(A, BL.gbad);
  auto* gsrc = at<int32_t>(A, BL.gsrc);
  auto* gdst = at<int32_t>(A, BL.gdst);
  auto* gw = at<uint32_t>(A, BL.gw);
  auto* cin = at<uint8_t>(A, BL.cin);
  auto* ctotal = at<uint64_t>(A, BL.total);
  auto* d_con = at<int32_t>(A, BL.con);
  auto* d_cpoff = at<int64_t>(A, BL.cpoff);
  auto* d_csoff = at<int64_t>(A, BL.csoff);
  auto* tot = reinterpret_cast<unsigned long long*>(total);

  HIP_OK(hipMemcpyAsync(d_voff, voff, 8 * ((size_t)G + 1), hipMemcpyHostToDevice, s));
  HIP_OK(hipMemcpyAsync(d_eoff, eoff, 8 * ((size_t)G + 1), hipMemcpyHostToDevice, s));
  if (!P.small.empty())
    HIP_OK(hipMemcpyAsync(d_small, P.small.data(), 4 * P.small.size(), hipMemcpyHostToDevice, s));
  if (!P.mid.empty()) HIP_OK(hipMemcpyAsync(d_mid, P.mid.data(), 4 * P.mid.size(), hipMemcpyHostToDevice, s));
  if (nuni > 0) {
    HIP_OK(hipMemcpyAsync(d_uni, P.uni.data(), 4 * (size_t)nuni, hipMemcpyHostToDevice, s));
    HIP_OK(hipMemcpyAsync(d_cvert, P.cvert.data(), 8 * P.cvert.size(), hipMemcpyHostToDevice, s));
    HIP_OK(hipMemcpyAsync(d_cedge, P.cedge.data(), 8 * P.cedge.size(), hipMemcpyHostToDevice, s));
    HIP_OK(hipMemsetAsync(d_gbad, 0, 4 * (size_t)nuni, s));
  }
  if (ncon > 0) {
    HIP_OK(hipMemcpyAsync(d_con, P.con.data(), 4 * (size_t)ncon, hipMemcpyHostToDevice, s));
    HIP_OK(hipMemcpyAsync(d_cpoff, P.cpoff.data(), 8 * (size_t)ncon, hipMemcpyHostToDevice, s));
    HIP_OK(hipMemcpyAsync(d_csoff, P.csoff.data(), 8 * (size_t)ncon, hipMemcpyHostToDevice, s));
  }
  if (eoff[G] > 0) HIP_OK(hipMemsetAsync(in_mst, 0, (size_t)eoff[G], s));
  HIP_OK(launch_one_workgroup_classes(P, BL, A, mid_limit, src, dst, w, in_mst, total, status, s));

  for (size_t c = 0; c + 1 < P.cfirst.size(); ++c) {
    const int32_t i0 = P.cfirst[c], ng = P.cfirst[c + 1] - i0;
    const int64_t at_meta = P.meta_at[c];
    const int64_t cn = P.cvert[at_meta + ng], cm = P.cedge[at_meta + ng];
    HIP_OK(launch_gather(d_uni + i0, ng, d_voff, d_eoff, d_cvert + at_meta, d_cedge + at_meta, cm, src, dst, w,
                         gsrc, gdst, gw, d_gbad + i0, s));
    if (cm > 0) {
      const Layout Lc = plan((int32_t)cn, cm);
      rc = solve_locked(dc, Lc, (int32_t)cn, cm, gsrc, gdst, gw, cin, ctotal, s);
      if (rc < 0) return rc;
    } else {
      HIP_OK(hipMemsetAsync(cin, 0, 1, s));
    }
    int64_t max_graph_m = 0;
    for (int32_t q = 0; q < ng; ++q)
      max_graph_m = std::max(max_graph_m, P.cedge[at_meta + q + 1] - P.cedge[at_meta + q]);
    HIP_OK(launch_graph_epilogue(d_uni + i0, ng, d_voff, d_eoff, d_cedge + at_meta, max_graph_m, cin, gw,
                                 d_gbad + i0, in_mst, at<unsigned long long>(A, BL.acc_w),
                                 at<uint32_t>(A, BL.acc_c), tot, status, s));
  }
  HIP_OK(hipStreamSynchronize(s));
  return MSTX_OK;
}

// A batch of fixed shape on fixed buffers, planned once and captured as a
// HIP graph: the flags cleared by a kernel (no memset node) and the
// one-launch solve of every graph.  Replays run the graph on any stream of
// the plan's device.
struct BatchGraphPlan {
  int device = 0;
  void* mem = nullptr;  // class lists, offsets and the contraction scratch (BatchLayout)
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

void plan_free(BatchGraphPlan* h) {
  if (h->exec) (void)hipGraphExecDestroy(h->exec);
  if (h->graph) (void)hipGraphDestroy(h->graph);
  if (h->mem) (void)hipFree(h->mem);
  delete h;
}

int batch_plan_create(int32_t G, const int64_t* voff, const int64_t* eoff, const int32_t* src, const int32_t* dst,
                      const uint32_t* w, uint8_t* in_mst, uint64_t* total, int32_t* status, hipStream_t s,
                      BatchGraphPlan** out) {
  *out = nullptr;
  const int32_t mid_limit = g_mid_limit.load();
  const BatchPlan P = plan_batch_graphs(G, voff, eoff, mid_limit);
  // graphs that need the union chunks' host-driven rounds cannot be captured
  if (!P.uni.empty()) return MSTX_ERR_INVALID_ARG;
  const BatchLayout BL = plan_batch(G, P);
  {
    // the kernels' LDS limits are raised once per device (as for a solve)
    DeviceCache* dc = nullptr;
    std::unique_lock<std::mutex> lock;
    const int rc = acquire(dc, lock, 0, s);
    if (rc != MSTX_OK) return rc;
  }
  std::unique_ptr<BatchGraphPlan, void (*)(BatchGraphPlan*)> h(new BatchGraphPlan(), plan_free);
  HIP_OK(hipGetDevice(&h->device));
  if (hipMalloc(&h->mem, std::max<size_t>(BL.bytes, 256)) != hipSuccess) {
    (void)hipGetLastError();
    h->mem = nullptr;
    return MSTX_ERR_OUT_OF_MEMORY;
  }
  void* A = h->mem;
  auto put = [&](size_t at_, const void* p, size_t bytes) {
    return bytes ? hipMemcpy(at<char>(A, at_), p, bytes, hipMemcpyHostToDevice) : hipSuccess;
  };
  HIP_OK(put(BL.voff, voff, 8 * ((size_t)G + 1)));
  HIP_OK(put(BL.eoff, eoff, 8 * ((size_t)G + 1)));
  HIP_OK(put(BL.small, P.small.data(), 4 * P.small.size()));
  HIP_OK(put(BL.mid, P.mid.data(), 4 * P.mid.size()));
  HIP_OK(put(BL.con, P.con.data(), 4 * P.con.size()));
  HIP_OK(put(BL.cpoff, P.cpoff.data(), 8 * P.cpoff.size()));
  HIP_OK(put(BL.csoff, P.csoff.data(), 8 * P.csoff.size()));
  // capture on a stream of our own (default priority), so that nothing the
  // caller enqueues meanwhile joins the graph
  hipStream_t cs = nullptr;
  HIP_OK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    hipError_t le = launch_fill_u8(in_mst, eoff[G], 0, cs);
    if (le == hipSuccess) le = launch_one_workgroup_classes(P, BL, A, mid_limit, src, dst, w, in_mst, total, status, cs);
    e = hipStreamEndCapture(cs, &h->graph);
    if (e == hipSuccess) e = le;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&h->exec, h->graph, nullptr, nullptr, 0);
  (void)hipStreamDestroy(cs);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return MSTX_ERR_DEVICE;
  }
  *out = h.release();
  return MSTX_OK;
}

int csr_to_edges(int32_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col, const uint32_t* w,
                 int32_t* out_src, int32_t* out_dst, uint32_t* out_w, int64_t* out_m, hipStream_t s) {
  const int64_t ntiles = csr_tiles(nnz);
  const size_t cnt_bytes = align_up(4 * (size_t)std::max<int64_t>(ntiles, 1));
  const size_t off_bytes = align_up(8 * (size_t)(ntiles + 1));
  DeviceCache* dc = nullptr;
  std::unique_lock<std::mutex> lock;
  int rc = acquire(dc, lock, 0, s);
  if (rc != MSTX_OK) return rc;
  rc = grow_aux(dc, cnt_bytes + off_bytes + 256, s);
  if (rc != MSTX_OK) return rc;
  auto* cnt = at<uint32_t>(dc->aux, 0);
  auto* off = at<int64_t>(dc->aux, cnt_bytes);
  auto* err = at<uint32_t>(dc->aux, cnt_bytes + off_bytes);
  HIP_OK(hipMemsetAsync(err, 0, sizeof(uint32_t), s));
  HIP_OK(launch_csr_to_edges(n, nnz, row_ptr, col, w, cnt, off, err, out_src, out_dst, out_w, s));
  uint32_t herr = 0;
  int64_t m = 0;
  HIP_OK(hipMemcpyAsync(&herr, err, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  if (ntiles > 0) HIP_OK(hipMemcpyAsync(&m, off + ntiles, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  if (herr & 1u) return MSTX_ERR_INVALID_ARG;
  if (herr & 2u) return MSTX_ERR_VERTEX_RANGE;
  if (m > (int64_t)0xFFFFFFFFLL) return MSTX_ERR_TOO_LARGE;
  *out_m = m;
  return MSTX_OK;
}

int select_min_edges(int32_t n, int64_t m, const int32_t* src, const int32_t* dst, const uint32_t* w,
                     uint64_t* out_best, hipStream_t s) {
  const Layout L = plan(n, m);
  if (L.bytes > workspace_limit()) return MSTX_ERR_OUT_OF_MEMORY;
  if (m > 0 && n == 0) return MSTX_ERR_VERTEX_RANGE;
  if (n == 0) return MSTX_OK;
  DeviceCache* dc = nullptr;
  std::unique_lock<std::mutex> lock;
  int rc = acquire(dc, lock, L.bytes, s);
  if (rc != MSTX_OK) return rc;
  void* B = dc->base;
  Solve S{};
  S.n = n;
  S.m = m;
  S.src = src;
  S.dst = dst;
  S.w = w;
  S.s = s;
  S.cus = dc->cus;
  S.rounds = dc->host_rounds;
  S.L = L;
  S.best = reinterpret_cast<unsigned long long*>(out_best);
  S.seg_cnt = at<uint32_t>(B, L.seg_cnt);
  S.seg_live = at<uint32_t>(B, L.seg_live);
  S.rec = at<uint4>(B, L.rec);
  S.labpool = at<int32_t>(B, L.labpool);
  S.st = at<DevState>(B, L.state);
  S.offers = L.bucket ? at<unsigned long long>(B, L.offers) : nullptr;
  S.offT = L.bucket ? at<uint32_t>(B, L.offT) : nullptr;
  S.slab = L.slab_cap ? at<unsigned long long>(B, L.slab) : nullptr;
  S.pbest = at<unsigned long long>(B, L.pbest);
  S.btot = at<uint32_t>(B, L.btot);
  S.dense_limit = 0;  // per-vertex minima: never the pair table
  S.bucket_limit = g_bucket_limit.load();
  S.in_mst = nullptr;
  t_timer.begin(s);
  t_timer.on = false;
  HIP_OK(launch_init(n, m, (int64_t)((L.cmap - L.labpool) / 4), 0, S.best, at<int32_t>(B, L.parent), nullptr,
                     S.btot, SparseTable{nullptr, nullptr, nullptr}, S.st, grid_for(n), s));
  if (m > 0) {
    hipError_t err = hipSuccess;
    enqueue_scan(S, 0, 0, n, true, err);
    HIP_OK(err);
  }
  int32_t err_flag = 0;
  HIP_OK(hipMemcpyAsync(&err_flag, &S.st->err, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  return err_flag ? MSTX_ERR_VERTEX_RANGE : MSTX_OK;
}

}  // namespace
}  // namespace mstx

extern "C" {

int mst_solve(int32_t n, int64_t m, const int32_t* src, const int32_t* dst, const uint32_t* w,
              uint8_t* out_in_mst, uint64_t* out_total_weight, void* stream) {
  int rc = mstx::check_args(n, m, src, dst, w);
  if (rc != MSTX_OK) return rc;
  if (!out_total_weight || (m > 0 && !out_in_mst)) return MSTX_ERR_INVALID_ARG;
  return mstx::solve(n, m, src, dst, w, out_in_mst, out_total_weight, (hipStream_t)stream);
}

int mst_solve_noalloc(int32_t n, int64_t m, const int32_t* src, const int32_t* dst, const uint32_t* w,
                      uint8_t* out_in_mst, uint64_t* out_total_weight, void* stream) {
  int rc = mstx::check_args(n, m, src, dst, w);
  if (rc != MSTX_OK) return rc;
  if (!out_total_weight || (m > 0 && !out_in_mst)) return MSTX_ERR_INVALID_ARG;
  return mstx::solve_noalloc(n, m, src, dst, w, out_in_mst, out_total_weight, (hipStream_t)stream);
}

int mst_solve_batched(int32_t num_graphs, const int64_t* vertex_offsets, const int64_t* edge_offsets,
                      const int32_t* src, const int32_t* dst, const uint32_t* w, uint8_t* out_in_mst,
                      uint64_t* out_total_weight, int32_t* out_status, void* stream) {
  int rc = mstx::check_batch_args(num_graphs, vertex_offsets, edge_offsets, src, dst, w, out_in_mst,
                                  out_total_weight, out_status);
  if (rc != MSTX_OK) return rc;
  return mstx::solve_batched(num_graphs, vertex_offsets, edge_offsets, src, dst, w, out_in_mst, out_total_weight,
                             out_status, (hipStream_t)stream);
}

size_t mst_batched_workspace_bytes(int32_t num_graphs, const int64_t* vertex_offsets, const int64_t* edge_offsets) {
  if (mstx::check_batch_args(num_graphs, vertex_offsets, edge_offsets, (void*)1, (void*)1, (void*)1, (void*)1,
                             (void*)1, (void*)1) != MSTX_OK)
    return 0;
  const mstx::BatchPlan P =
      mstx::plan_batch_graphs(num_graphs, vertex_offsets, edge_offsets, mstx::g_mid_limit.load());
  const size_t solve_ws =
      P.uni.empty() ? 0 : mstx::plan((int32_t)std::min<int64_t>(P.max_chunk_n, INT32_MAX), P.max_chunk_m).bytes;
  return solve_ws + mstx::plan_batch(num_graphs, P).bytes;
}

int mst_csr_to_edges(int32_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col, const uint32_t* w,
                     int32_t* out_src, int32_t* out_dst, uint32_t* out_w, int64_t* out_m, void* stream) {
  if (n < 0 || nnz < 0 || !row_ptr || !out_m) return MSTX_ERR_INVALID_ARG;
  if (nnz > 0 && (!col || !w || !out_src || !out_dst || !out_w)) return MSTX_ERR_INVALID_ARG;
  return mstx::csr_to_edges(n, nnz, row_ptr, col, w, out_src, out_dst, out_w, out_m, (hipStream_t)stream);
}

int mst_select_min_edges(int32_t n, int64_t m, const int32_t* src, const int32_t* dst, const uint32_t* w,
                         uint64_t* out_best, void* stream) {
  int rc = mstx::check_args(n, m, src, dst, w);
  if (rc != MSTX_OK) return rc;
  if (n > 0 && !out_best) return MSTX_ERR_INVALID_ARG;
  return mstx::select_min_edges(n, m, src, dst, w, out_best, (hipStream_t)stream);
}

int mst_last_round_stats(int64_t* out, int32_t max_rounds) {
  if (max_rounds < 0 || (max_rounds > 0 && !out)) return MSTX_ERR_INVALID_ARG;
  const int k = std::min(mstx::t_last_stats.rounds, (int)max_rounds);
  if (k > 0) std::memcpy(out, mstx::t_last_stats.v, sizeof(int64_t) * 3 * (size_t)k);
  return k;
}

int mst_profile_enable(int enable) {
  std::lock_guard<std::mutex> g(mstx::g_prof.mu);
  const int was = mstx::g_prof.enabled ? 1 : 0;
  mstx::g_prof.enabled = enable != 0;
  if (enable) mstx::g_prof.clear();
  return was;
}

int mst_profile_read(double* out_ms, int64_t* out_launches, double* out_bytes, int32_t kinds) {
  if (kinds < 0 || (kinds > 0 && (!out_ms || !out_launches || !out_bytes))) return MSTX_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> g(mstx::g_prof.mu);
  const int k = std::min<int>(kinds, mstx::kKinds);
  for (int i = 0; i < k; ++i) {
    out_ms[i] = mstx::g_prof.ms[i];
    out_launches[i] = mstx::g_prof.launches[i];
    out_bytes[i] = mstx::g_prof.bytes[i];
  }
  return mstx::kKinds;
}

int mst_profile_read_rounds(double* out_ms, int64_t* out_launches, double* out_bytes, int32_t max_rounds) {
  if (max_rounds < 0 || (max_rounds > 0 && (!out_ms || !out_launches || !out_bytes))) return MSTX_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> g(mstx::g_prof.mu);
  const int rows = std::min<int>(max_rounds, mstx::kMaxRounds + 1);
  for (int r = 0; r < rows; ++r)
    for (int k = 0; k < mstx::kKinds; ++k) {
      out_ms[(size_t)r * mstx::kKinds + k] = mstx::g_prof.rms[r][k];
      out_launches[(size_t)r * mstx::kKinds + k] = mstx::g_prof.rlaunches[r][k];
      out_bytes[(size_t)r * mstx::kKinds + k] = mstx::g_prof.rbytes[r][k];
    }
  return mstx::kKinds;
}

const char* mst_profile_kernel_name(int kind) {
  return (kind >= 0 && kind < mstx::kKinds) ? mstx::kKindNames[kind] : "";
}

int mst_workspace_release(void* stream) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return MSTX_ERR_DEVICE;
  std::unique_ptr<mstx::DeviceCache> victim;
  {
    std::lock_guard<std::mutex> g(mstx::g_caches_mu);
    auto it = mstx::g_caches.find({dev, (hipStream_t)stream});
    if (it == mstx::g_caches.end()) return MSTX_OK;
    std::lock_guard<std::mutex> l(it->second->mu);  // no call of this stream is running
    if (it->second->step_active) return MSTX_ERR_INVALID_ARG;  // a stepwise solve still owns its workspace
    victim = std::move(it->second);
    mstx::g_caches.erase(it);
  }
  // the workspace and the batched scratch are stream-ordered allocations
  if (victim->base && hipFreeAsync(victim->base, (hipStream_t)stream) != hipSuccess) return MSTX_ERR_DEVICE;
  if (victim->aux && hipFreeAsync(victim->aux, (hipStream_t)stream) != hipSuccess) return MSTX_ERR_DEVICE;
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return MSTX_ERR_DEVICE;
  if (victim->host_rounds && hipHostFree(victim->host_rounds) != hipSuccess) return MSTX_ERR_DEVICE;
  if (victim->small_dev && hipFree(victim->small_dev) != hipSuccess) return MSTX_ERR_DEVICE;
  if (victim->small_host && hipHostFree(victim->small_host) != hipSuccess) return MSTX_ERR_DEVICE;
  for (auto& e : victim->round_ev)
    if (e) (void)hipEventDestroy(e);
  if (victim->step_base && hipFree(victim->step_base) != hipSuccess) return MSTX_ERR_DEVICE;
  if (victim->step_rounds && hipHostFree(victim->step_rounds) != hipSuccess) return MSTX_ERR_DEVICE;
  for (auto& e : victim->step_ev)
    if (e) (void)hipEventDestroy(e);
  return MSTX_OK;
}

int mst_solve_begin(int32_t n, int64_t m, const int32_t* src, const int32_t* dst, const uint32_t* w,
                    uint8_t* out_in_mst, uint64_t* out_total_weight, void* stream, MstxSolve** out_handle) {
  if (!out_handle) return MSTX_ERR_INVALID_ARG;
  *out_handle = nullptr;
  int rc = mstx::check_args(n, m, src, dst, w);
  if (rc != MSTX_OK) return rc;
  if (!out_total_weight || (m > 0 && !out_in_mst)) return MSTX_ERR_INVALID_ARG;
  mstx::StepSolve* h = nullptr;
  rc = mstx::step_begin(n, m, src, dst, w, out_in_mst, out_total_weight, (hipStream_t)stream, &h);
  *out_handle = reinterpret_cast<MstxSolve*>(h);
  return rc;
}

int mst_solve_advance(MstxSolve* handle, int32_t* out_done) {
  if (!handle || !out_done) return MSTX_ERR_INVALID_ARG;
  auto* h = reinterpret_cast<mstx::StepSolve*>(handle);
  mstx::step_advance(h, false);
  *out_done = h->done ? 1 : 0;
  return MSTX_OK;
}

int mst_solve_wait_round(MstxSolve* handle, int32_t* out_done) {
  if (!handle || !out_done) return MSTX_ERR_INVALID_ARG;
  auto* h = reinterpret_cast<mstx::StepSolve*>(handle);
  mstx::step_advance(h, true, true);
  *out_done = h->done ? 1 : 0;
  return MSTX_OK;
}

int mst_solve_end(MstxSolve* handle) {
  if (!handle) return MSTX_ERR_INVALID_ARG;
  auto* h = reinterpret_cast<mstx::StepSolve*>(handle);
  mstx::step_advance(h, true);
  const int st = h->status;
  delete h;
  return st;
}

int mst_batched_plan_create(int32_t num_graphs, const int64_t* vertex_offsets, const int64_t* edge_offsets,
                            const int32_t* src, const int32_t* dst, const uint32_t* w, uint8_t* out_in_mst,
                            uint64_t* out_total_weight, int32_t* out_status, void* stream, MstxBatchPlan** out_plan) {
  if (!out_plan) return MSTX_ERR_INVALID_ARG;
  *out_plan = nullptr;
  if (num_graphs <= 0) return MSTX_ERR_INVALID_ARG;
  int rc = mstx::check_batch_args(num_graphs, vertex_offsets, edge_offsets, src, dst, w, out_in_mst, out_total_weight,
                                  out_status);
  if (rc != MSTX_OK) return rc;
  mstx::BatchGraphPlan* h = nullptr;
  rc = mstx::batch_plan_create(num_graphs, vertex_offsets, edge_offsets, src, dst, w, out_in_mst, out_total_weight,
                               out_status, (hipStream_t)stream, &h);
  if (rc != MSTX_OK) return rc;
  *out_plan = reinterpret_cast<MstxBatchPlan*>(h);
  return MSTX_OK;
}

int mst_batched_plan_run(MstxBatchPlan* plan, void* stream) {
  if (!plan) return MSTX_ERR_INVALID_ARG;
  auto* h = reinterpret_cast<mstx::BatchGraphPlan*>(plan);
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != h->device) return MSTX_ERR_INVALID_ARG;
  return hipGraphLaunch(h->exec, (hipStream_t)stream) == hipSuccess ? MSTX_OK : MSTX_ERR_DEVICE;
}

int mst_batched_plan_destroy(MstxBatchPlan* plan) {
  if (!plan) return MSTX_ERR_INVALID_ARG;
  mstx::plan_free(reinterpret_cast<mstx::BatchGraphPlan*>(plan));
  return MSTX_OK;
}

size_t mst_workspace_bytes(int32_t n, int64_t m) {
  if (n < 0 || m < 0 || m > (int64_t)0xFFFFFFFFLL) return 0;
  return mstx::plan(n, m).bytes;
}

int32_t mst_set_small_limit(int32_t limit) {
  if (limit < 0) return mstx::g_small_limit.load();
  return mstx::g_small_limit.exchange(std::min<int32_t>(limit, mstx::kSmallN));
}

int32_t mst_set_mid_limit(int32_t limit) {
  if (limit < 0) return mstx::g_mid_limit.load();
  return mstx::g_mid_limit.exchange(std::min<int32_t>(limit, mstx::kMidN));
}

int32_t mst_set_tail_limit(int32_t limit) {
  if (limit < 0) return mstx::g_tail_limit.load();
  return mstx::g_tail_limit.exchange(std::min<int32_t>(limit, mstx::kTailMax));
}

int32_t mst_set_bucket_limit(int32_t limit) {
  if (limit < 0) return (int32_t)mstx::g_bucket_limit.load();
  return (int32_t)mstx::g_bucket_limit.exchange(std::min<int64_t>(limit, mstx::kBucketMaxComponents));
}

int32_t mst_set_sparse_limit(int32_t live_edges) {
  if (live_edges < 0) return mstx::g_sparse_limit.load();
  return mstx::g_sparse_limit.exchange(live_edges);
}

int32_t mst_set_scan_occupancy(int32_t wg_per_cu) {
  if (wg_per_cu < 0) return mstx::g_scan_occupancy.load();
  return mstx::g_scan_occupancy.exchange(std::min<int32_t>(wg_per_cu, 8));
}

int32_t mst_set_dense_limit(int32_t limit) {
  if (limit < 0) return mstx::g_dense_limit.load();
  return mstx::g_dense_limit.exchange(std::min<int32_t>(limit, mstx::kDenseMax));
}

const char* mst_status_string(int status) {
  switch (status) {
    case MSTX_OK: return "ok: minimum spanning tree";
    case MSTX_DISCONNECTED: return "ok: graph is disconnected, result is the minimum spanning forest";
    case MSTX_ERR_INVALID_ARG: return "invalid argument (negative size or NULL array)";
    case MSTX_ERR_VERTEX_RANGE: return "an edge end point is outside [0, n)";
    case MSTX_ERR_TOO_LARGE: return "too many edges: m must be <= 0xFFFFFFFF";
    case MSTX_ERR_OUT_OF_MEMORY: return "device workspace allocation failed or exceeds MSTX_WORKSPACE_LIMIT_BYTES";
    case MSTX_ERR_DEVICE: return "HIP runtime error or round-count watchdog";
    case MSTX_ERR_SCRATCH_LIMIT:
      return "graph too large for mst_solve_noalloc: its workspace (mst_workspace_bytes) plus 2 KB of round "
             "records must fit the library's fixed 256 MiB device scratch";
    default: return "unknown status";
  }
}

}  // extern "C"
