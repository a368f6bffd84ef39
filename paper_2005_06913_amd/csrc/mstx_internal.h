// mstx_internal.h -- declarations shared by the kernels and the host driver.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mstx {

// No edge: larger than every real key ((w << 32) | e with e <= 0xFFFFFFFE).
static constexpr unsigned long long kKeyNone = ~0ull;

// Upper bound on rounds recorded: the number of components with an outgoing
// edge at least halves every round, so ceil(log2 n) + 1 <= 33 for int32 n.
static constexpr int kMaxRounds = 40;

// Device-resident round state.  Round r's kernels read n[r] and lab_off[r];
// the finalize kernel of round r writes n[r+1], lab_off[r+1], live[r], sel[r].
struct DevState {
  int32_t n[kMaxRounds + 1];        // components entering round r (isolated ones dropped)
  int64_t lab_off[kMaxRounds + 1];  // offset of round r's label map in the label pool
  int64_t live[kMaxRounds];         // edges between different components at round r
  int64_t sel[kMaxRounds];          // edges added in round r
  int64_t edges_added;              // running total of sel[]
  int32_t err;                      // an edge end outside [0, n) was seen
  int32_t err_internal;             // a label lookup gave an impossible value
};

hipError_t launch_init(int32_t n, uint32_t m, unsigned long long* best, int32_t* parent, DevState* st,
                       int grid, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long* p, int64_t count, unsigned long long v, int grid,
                           hipStream_t s);
hipError_t launch_scan_first(bool lds, const int32_t* src, const int32_t* dst, const uint32_t* w,
                             uint32_t m, int32_t n, unsigned long long* best, uint32_t* part_live,
                             DevState* st, int grid, hipStream_t s);
hipError_t launch_scan_seg(bool from_input, bool lds, int32_t nr_host, int round, const int32_t* src,
                           const int32_t* dst, const uint32_t* w, uint32_t m, const int32_t* labpool,
                           uint4* rec, uint32_t* seg_cnt, uint32_t seg_cap, int32_t nseg,
                           unsigned long long* best, const DevState* st, int grid, hipStream_t s);
hipError_t launch_hook(int round, const int32_t* src, const int32_t* dst, const uint32_t* w,
                       const unsigned long long* best, int32_t* parent, const int32_t* labpool,
                       DevState* st, uint8_t* in_mst, uint32_t* part_sel,
                       unsigned long long* part_w, int grid, hipStream_t s);
hipError_t launch_compress(int round, int32_t* parent, int32_t* root_of, const unsigned long long* best,
                           unsigned long long* rootmask, int32_t* rootcnt, const DevState* st, int grid,
                           hipStream_t s);
hipError_t launch_finalize(int round, const int32_t* rootcnt, int32_t* rootpre, const uint32_t* part_live,
                           int32_t nlive, const uint32_t* part_sel, const unsigned long long* part_w,
                           int32_t nhook, DevState* st, unsigned long long* total, hipStream_t s);
hipError_t launch_relabel(int round, const int32_t* root_of, const unsigned long long* rootmask,
                          const int32_t* rootpre, int32_t* labpool, int32_t* parent,
                          unsigned long long* best, const DevState* st, int grid, hipStream_t s);

}  // namespace mstx
