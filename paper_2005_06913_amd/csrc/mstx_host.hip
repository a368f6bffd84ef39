// mstx_host.hip -- host driver and C ABI of the parallel Boruvka MST.
//
// Argument checks run on the host before any HIP call.  The workspace (all
// device scratch) is planned from (n, m), cached per device and guarded by a
// mutex.  The round loop enqueues the five kernels of a round on the caller's
// stream and reads back the 1 KB round state to decide whether another round
// is needed.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

#include "mstx.h"
#include "mstx_internal.h"

namespace mstx {
namespace {

constexpr int kBlockThreads = 256;
constexpr int kMaxGrid = 4096;        // capacity of the per-block partial arrays
constexpr int kMaxSegments = 2048;    // segments of the record stream
constexpr uint32_t kMinSegment = 1024;
constexpr int32_t kLdsSlots = 8192;   // per-workgroup minima kept in LDS (64 KiB)

struct Layout {
  size_t best, parent, root_of, labpool, rootmask, rootcnt, rootpre, rec, seg_cnt, part_live, part_sel,
      part_w, state, bytes;
  int32_t nseg;
  uint32_t seg_cap;
};

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

// Workspace plan for a graph with n vertices and m edges.
Layout plan(int32_t n, int64_t m) {
  Layout L{};
  const size_t N = (size_t)std::max<int32_t>(n, 1);
  const size_t words = (N + 63) / 64 + 1;
  int64_t nseg = (m + kMinSegment - 1) / kMinSegment;
  nseg = std::max<int64_t>(1, std::min<int64_t>(nseg, kMaxSegments));
  const uint64_t seg_cap = m > 0 ? (uint64_t)((m + nseg - 1) / nseg) : 1;
  L.nseg = (int32_t)nseg;
  L.seg_cap = (uint32_t)seg_cap;
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
  L.rootmask = take(8 * words);
  L.rootcnt = take(4 * words);
  L.rootpre = take(4 * words);
  L.rec = take(16 * (size_t)nseg * seg_cap);
  L.seg_cnt = take(4 * (size_t)nseg);
  L.part_live = take(4 * (size_t)kMaxGrid);
  L.part_sel = take(4 * (size_t)kMaxGrid);
  L.part_w = take(8 * (size_t)kMaxGrid);
  L.state = take(sizeof(DevState));
  L.bytes = off;
  return L;
}

struct DeviceCache {
  std::mutex mu;
  void* base = nullptr;
  size_t bytes = 0;
  DevState* host_state = nullptr;  // pinned
  int cus = 0;
};

constexpr int kMaxDevices = 64;
DeviceCache g_dev[kMaxDevices];

thread_local std::vector<int64_t> t_last_stats;

// ------------------------------------------------------------- profiling
// Opt-in per-kernel timing: when enabled, every kernel launch of a solve is
// bracketed by two hipEvents on the solve's stream.  After the solve the
// elapsed times are accumulated per kernel kind together with the kind's
// algorithmic bytes (bytes the method must move, computed from the round
// statistics).
enum Kind { kScanFirst = 0, kScanInput, kScanRecords, kHook, kCompress, kFinalize, kRelabel, kKinds };
const char* const kKindNames[kKinds] = {"scan_first", "scan_input", "scan_records", "hook",
                                        "compress",   "finalize",   "relabel"};

struct Profile {
  std::mutex mu;
  bool enabled = false;
  double ms[kKinds] = {};
  int64_t launches[kKinds] = {};
  double bytes[kKinds] = {};
};
Profile g_prof;

struct PendingLaunch {
  int kind;
  hipEvent_t a, b;
  double bytes;
};

// Events of one solve; reused across solves on this thread.
struct LaunchTimer {
  bool on = false;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  std::vector<PendingLaunch> pending;
  hipStream_t s = nullptr;

  hipError_t begin(hipStream_t stream) {
    on = false;
    {
      std::lock_guard<std::mutex> g(g_prof.mu);
      on = g_prof.enabled;
    }
    used = 0;
    pending.clear();
    s = stream;
    return hipSuccess;
  }
  hipError_t event(hipEvent_t* out) {
    if (used == pool.size()) {
      hipEvent_t e;
      hipError_t r = hipEventCreate(&e);
      if (r != hipSuccess) return r;
      pool.push_back(e);
    }
    *out = pool[used++];
    return hipSuccess;
  }
  // Records the start event; returns the pending slot (or -1 when off).
  int start(int kind) {
    if (!on) return -1;
    PendingLaunch p{kind, nullptr, nullptr, 0.0};
    if (event(&p.a) != hipSuccess || event(&p.b) != hipSuccess) return -1;
    if (hipEventRecord(p.a, s) != hipSuccess) return -1;
    pending.push_back(p);
    return (int)pending.size() - 1;
  }
  void stop(int slot, double bytes = 0.0) {
    if (slot < 0) return;
    pending[slot].bytes = bytes;
    (void)hipEventRecord(pending[slot].b, s);
  }
  void set_bytes(int slot, double bytes) {
    if (slot >= 0) pending[slot].bytes = bytes;
  }
  // Call after the stream has been synchronised.
  void commit() {
    if (!on) return;
    std::lock_guard<std::mutex> g(g_prof.mu);
    for (const auto& p : pending) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, p.a, p.b) != hipSuccess) continue;
      g_prof.ms[p.kind] += ms;
      g_prof.launches[p.kind] += 1;
      g_prof.bytes[p.kind] += p.bytes;
    }
    pending.clear();
  }
};
thread_local LaunchTimer t_timer;

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

#define HIP_OK(expr)                              \
  do {                                            \
    if ((expr) != hipSuccess) return MSTX_ERR_DEVICE; \
  } while (0)

// Locks the device cache, grows the workspace to `bytes`.
int acquire(DeviceCache*& dc, std::unique_lock<std::mutex>& lock, size_t bytes) {
  int dev = 0;
  HIP_OK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return MSTX_ERR_DEVICE;
  dc = &g_dev[dev];
  lock = std::unique_lock<std::mutex>(dc->mu);
  if (!dc->host_state) {
    HIP_OK(hipHostMalloc((void**)&dc->host_state, sizeof(DevState), hipHostMallocDefault));
    hipDeviceProp_t prop;
    HIP_OK(hipGetDeviceProperties(&prop, dev));
    dc->cus = prop.multiProcessorCount;
  }
  if (dc->bytes < bytes) {
    if (dc->base) {
      HIP_OK(hipDeviceSynchronize());
      HIP_OK(hipFree(dc->base));
      dc->base = nullptr;
      dc->bytes = 0;
    }
    if (hipMalloc(&dc->base, bytes) != hipSuccess) {
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
  int rc = acquire(dc, lock, L.bytes);
  if (rc != MSTX_OK) return rc;
  void* B = dc->base;
  auto* best = at<unsigned long long>(B, L.best);
  auto* parent = at<int32_t>(B, L.parent);
  auto* root_of = at<int32_t>(B, L.root_of);
  auto* labpool = at<int32_t>(B, L.labpool);
  auto* rootmask = at<unsigned long long>(B, L.rootmask);
  auto* rootcnt = at<int32_t>(B, L.rootcnt);
  auto* rootpre = at<int32_t>(B, L.rootpre);
  auto* rec = at<uint4>(B, L.rec);
  auto* seg_cnt = at<uint32_t>(B, L.seg_cnt);
  auto* part_live = at<uint32_t>(B, L.part_live);
  auto* part_sel = at<uint32_t>(B, L.part_sel);
  auto* part_w = at<unsigned long long>(B, L.part_w);
  auto* st = at<DevState>(B, L.state);
  auto* tot = reinterpret_cast<unsigned long long*>(total);
  DevState* hs = dc->host_state;
  const uint32_t mu = (uint32_t)m;

  HIP_OK(hipMemsetAsync(in_mst, 0, (size_t)m, s));
  HIP_OK(hipMemsetAsync(total, 0, sizeof(uint64_t), s));
  HIP_OK(launch_init(n, mu, best, parent, st, grid_for(n), s));

  const int max_rounds = std::min(rounds_bound(n) + 1, kMaxRounds);
  LaunchTimer& T = t_timer;
  T.begin(s);
  int32_t nr = n;
  int64_t live_prev = 0;
  int rounds = 0;
  bool done = false;
  for (int r = 0; r < max_rounds && !done; ++r) {
    int nlive;
    const uint32_t* live_parts;
    int scan_slot;
    if (r == 0) {
      const bool lds = n <= kLdsSlots;
      const int g = lds ? std::min(grid_for(m), 2 * dc->cus) : grid_for(m);
      scan_slot = T.start(kScanFirst);
      HIP_OK(launch_scan_first(lds, src, dst, w, mu, n, best, part_live, st, g, s));
      T.stop(scan_slot);
      nlive = g;
      live_parts = part_live;
    } else {
      const bool lds = nr <= kLdsSlots;
      const int g = lds ? std::min(L.nseg, 2 * dc->cus) : L.nseg;
      scan_slot = T.start(r == 1 ? kScanInput : kScanRecords);
      HIP_OK(launch_scan_seg(r == 1, lds, nr, r, src, dst, w, mu, labpool, rec, seg_cnt, L.seg_cap, L.nseg,
                             best, st, g, s));
      T.stop(scan_slot);
      nlive = L.nseg;
      live_parts = seg_cnt;
    }
    const int gh = grid_for(nr);
    int k = T.start(kHook);
    HIP_OK(launch_hook(r, src, dst, w, best, parent, labpool, st, in_mst, part_sel, part_w, gh, s));
    T.stop(k);
    k = T.start(kCompress);
    HIP_OK(launch_compress(r, parent, root_of, best, rootmask, rootcnt, st, gh, s));
    T.stop(k);
    k = T.start(kFinalize);
    HIP_OK(launch_finalize(r, rootcnt, rootpre, live_parts, nlive, part_sel, part_w, gh, st, tot, s));
    T.stop(k);
    k = T.start(kRelabel);
    HIP_OK(launch_relabel(r, root_of, rootmask, rootpre, labpool, parent, best, st, gh, s));
    T.stop(k);
    HIP_OK(hipMemcpyAsync(hs, st, sizeof(DevState), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    rounds = r + 1;
    if (r == 0 && hs->err) return MSTX_ERR_VERTEX_RANGE;
    if (hs->err_internal) return MSTX_ERR_DEVICE;
    // algorithmic bytes of this round's scan: the edge stream read once, the
    // previous label map read once, best[] initialised and written once, the
    // compacted survivors written once
    const double nrd = (double)nr, live_r = (double)hs->live[r];
    double b;
    if (r == 0) b = 12.0 * (double)m + 16.0 * nrd;
    else if (r == 1) b = 12.0 * (double)m + 4.0 * (double)n + 16.0 * nrd + 16.0 * live_r;
    else b = 16.0 * (double)live_prev + 4.0 * (double)hs->n[r - 1] + 16.0 * nrd + 16.0 * live_r;
    T.set_bytes(scan_slot, b);
    live_prev = hs->live[r];
    nr = hs->n[r + 1];
    if (nr <= 1) done = true;
  }
  T.commit();
  if (!done) return MSTX_ERR_DEVICE;  // more rounds than the halving bound allows
  t_last_stats.resize(3 * (size_t)rounds);
  for (int r = 0; r < rounds; ++r) {
    t_last_stats[3 * r + 0] = hs->n[r];
    t_last_stats[3 * r + 1] = hs->live[r];
    t_last_stats[3 * r + 2] = hs->sel[r];
  }
  return (n <= 1 || hs->edges_added == (int64_t)n - 1) ? MSTX_OK : MSTX_DISCONNECTED;
}

int select_min_edges(int32_t n, int64_t m, const int32_t* src, const int32_t* dst, const uint32_t* w,
                     uint64_t* out_best, hipStream_t s) {
  const Layout L = plan(n, m);
  if (L.bytes > workspace_limit()) return MSTX_ERR_OUT_OF_MEMORY;
  if (m > 0 && n == 0) return MSTX_ERR_VERTEX_RANGE;
  if (n == 0) return MSTX_OK;
  DeviceCache* dc = nullptr;
  std::unique_lock<std::mutex> lock;
  int rc = acquire(dc, lock, L.bytes);
  if (rc != MSTX_OK) return rc;
  void* B = dc->base;
  auto* part_live = at<uint32_t>(B, L.part_live);
  auto* st = at<DevState>(B, L.state);
  auto* best = reinterpret_cast<unsigned long long*>(out_best);
  HIP_OK(launch_init(0, (uint32_t)m, best, at<int32_t>(B, L.parent), st, 1, s));
  HIP_OK(launch_fill_u64(best, n, kKeyNone, grid_for(n), s));
  if (m > 0) {
    const bool lds = n <= kLdsSlots;
    const int g = lds ? std::min(grid_for(m), 2 * dc->cus) : grid_for(m);
    HIP_OK(launch_scan_first(lds, src, dst, w, (uint32_t)m, n, best, part_live, st, g, s));
  }
  HIP_OK(hipMemcpyAsync(dc->host_state, st, sizeof(DevState), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  return dc->host_state->err ? MSTX_ERR_VERTEX_RANGE : MSTX_OK;
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

int mst_select_min_edges(int32_t n, int64_t m, const int32_t* src, const int32_t* dst, const uint32_t* w,
                         uint64_t* out_best, void* stream) {
  int rc = mstx::check_args(n, m, src, dst, w);
  if (rc != MSTX_OK) return rc;
  if (n > 0 && !out_best) return MSTX_ERR_INVALID_ARG;
  return mstx::select_min_edges(n, m, src, dst, w, out_best, (hipStream_t)stream);
}

int mst_last_round_stats(int64_t* out, int32_t max_rounds) {
  if (max_rounds < 0 || (max_rounds > 0 && !out)) return MSTX_ERR_INVALID_ARG;
  const int have = (int)(mstx::t_last_stats.size() / 3);
  const int k = std::min(have, (int)max_rounds);
  if (k > 0) std::memcpy(out, mstx::t_last_stats.data(), sizeof(int64_t) * 3 * (size_t)k);
  return k;
}

int mst_profile_enable(int enable) {
  std::lock_guard<std::mutex> g(mstx::g_prof.mu);
  const int was = mstx::g_prof.enabled ? 1 : 0;
  mstx::g_prof.enabled = enable != 0;
  if (enable) {
    for (int k = 0; k < mstx::kKinds; ++k) {
      mstx::g_prof.ms[k] = 0.0;
      mstx::g_prof.launches[k] = 0;
      mstx::g_prof.bytes[k] = 0.0;
    }
  }
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

const char* mst_profile_kernel_name(int kind) {
  return (kind >= 0 && kind < mstx::kKinds) ? mstx::kKindNames[kind] : "";
}

size_t mst_workspace_bytes(int32_t n, int64_t m) {
  if (n < 0 || m < 0 || m > (int64_t)0xFFFFFFFFLL) return 0;
  return mstx::plan(n, m).bytes;
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
    default: return "unknown status";
  }
}

}  // extern "C"
