// mstx_csr.hip -- the edge list of a symmetric CSR adjacency.
//
// The solve takes an edge list (Section 2.1's input graph, each undirected
// edge once).  A graph held as a symmetric adjacency structure (CSR: the arcs
// of vertex u are col[row_ptr[u] .. row_ptr[u+1]), every edge stored as the
// two arcs u -> v and v -> u) becomes one by keeping each arc with u < v, in
// row-major arc order; the mirrored copies (u > v) and self-loops (u == v)
// are dropped.  Three kernels: the arcs kept per tile, an exclusive scan of
// the tile counts, and the stable scatter of the kept arcs.  The row_ptr and
// column checks set bits of an error word instead of trapping, and no access
// depends on row_ptr being valid, so an invalid adjacency is reported, not
// read out of bounds.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <stdint.h>

#include "mstx.h"
#include "mstx_internal.h"

namespace mstx {

static constexpr int kCsrBlock = 256;
static constexpr int kCsrPer = 16;  // consecutive arcs per thread
static constexpr int64_t kCsrTile = (int64_t)kCsrBlock * kCsrPer;

// The row of arc a: the last u with row_ptr[u] <= a (rows may be empty).
// Stays in [0, n) whatever row_ptr holds.
__device__ __forceinline__ int32_t csr_row(const int64_t* __restrict__ row_ptr, int32_t n, int64_t a) {
  int32_t lo = 0, hi = n;
  while (hi - lo > 1) {
    const int32_t mid = lo + (hi - lo) / 2;
    if (row_ptr[mid] <= a) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Exclusive prefix sum over the kCsrBlock threads; *total gets the sum.
__device__ __forceinline__ uint32_t csr_block_scan(uint32_t v, uint32_t* wsum /* [kCsrBlock / 64] */,
                                                   uint32_t* total) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint32_t x = v;
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) wsum[wv] = x;
  __syncthreads();
  uint32_t before = 0, all = 0;
  for (int i = 0; i < kCsrBlock / 64; ++i) {
    if (i < wv) before += wsum[i];
    all += wsum[i];
  }
  *total = all;
  return before + x - v;
}

// err |= 1: row_ptr[0] != 0, row_ptr[n] != nnz or a decreasing step.
__global__ void __launch_bounds__(kCsrBlock) k_csr_check_rows(int32_t n, int64_t nnz,
                                                              const int64_t* __restrict__ row_ptr,
                                                              uint32_t* __restrict__ err) {
  const int64_t stride = (int64_t)gridDim.x * kCsrBlock;
  for (int64_t u = (int64_t)blockIdx.x * kCsrBlock + threadIdx.x; u < n; u += stride)
    if (row_ptr[u] > row_ptr[u + 1]) atomicOr(err, 1u);
  if (blockIdx.x == 0 && threadIdx.x == 0 && (row_ptr[0] != 0 || row_ptr[n] != nnz)) atomicOr(err, 1u);
}

// Whether arc a is kept (u < v); bad = 1 for a column outside [0, n) (err |= 2).
__device__ __forceinline__ bool csr_keep(const int64_t* row_ptr, const int32_t* col, int32_t n, int64_t a,
                                         int32_t& u, int32_t& v, uint32_t& bad) {
  v = col[a];
  if ((uint32_t)v >= (uint32_t)n) {
    bad = 1;
    return false;
  }
  u = csr_row(row_ptr, n, a);
  return u < v;
}

// cnt[t] = arcs kept in tile t (thread i of the tile owns kCsrPer consecutive arcs).
__global__ void __launch_bounds__(kCsrBlock) k_csr_count(int32_t n, int64_t nnz, const int64_t* __restrict__ row_ptr,
                                                         const int32_t* __restrict__ col,
                                                         uint32_t* __restrict__ cnt, uint32_t* __restrict__ err) {
  __shared__ uint32_t wsum[kCsrBlock / 64];
  const int64_t a0 = (int64_t)blockIdx.x * kCsrTile + (int64_t)threadIdx.x * kCsrPer;
  uint32_t kept = 0, bad = 0;
  for (int k = 0; k < kCsrPer; ++k) {
    const int64_t a = a0 + k;
    if (a >= nnz) break;
    int32_t u, v;
    if (csr_keep(row_ptr, col, n, a, u, v, bad)) ++kept;
  }
  if (bad) atomicOr(err, 2u);
  uint32_t total = 0;
  (void)csr_block_scan(kept, wsum, &total);
  if (threadIdx.x == 0) cnt[blockIdx.x] = total;
}

// off[t] = sum of cnt[0 .. t); off[ntiles] = the total.  One workgroup.
__global__ void __launch_bounds__(kCsrBlock) k_csr_scan(int64_t ntiles, const uint32_t* __restrict__ cnt,
                                                        int64_t* __restrict__ off) {
  __shared__ uint32_t wsum[kCsrBlock / 64];
  int64_t carry = 0;
  for (int64_t t0 = 0; t0 < ntiles; t0 += kCsrBlock) {
    const int64_t t = t0 + threadIdx.x;
    const uint32_t c = t < ntiles ? cnt[t] : 0u;
    uint32_t total = 0;
    const uint32_t before = csr_block_scan(c, wsum, &total);
    if (t < ntiles) off[t] = carry + before;
    carry += total;
    __syncthreads();  // wsum is rewritten by the next chunk
  }
  if (threadIdx.x == 0) off[ntiles] = carry;
}

// The kept arcs of tile t, in arc order, from position off[t].
__global__ void __launch_bounds__(kCsrBlock) k_csr_scatter(int32_t n, int64_t nnz,
                                                           const int64_t* __restrict__ row_ptr,
                                                           const int32_t* __restrict__ col,
                                                           const uint32_t* __restrict__ w,
                                                           const int64_t* __restrict__ off,
                                                           int32_t* __restrict__ out_src,
                                                           int32_t* __restrict__ out_dst,
                                                           uint32_t* __restrict__ out_w) {
  __shared__ uint32_t wsum[kCsrBlock / 64];
  const int64_t a0 = (int64_t)blockIdx.x * kCsrTile + (int64_t)threadIdx.x * kCsrPer;
  uint32_t kept = 0, bad = 0;
  for (int k = 0; k < kCsrPer; ++k) {
    const int64_t a = a0 + k;
    if (a >= nnz) break;
    int32_t u, v;
    if (csr_keep(row_ptr, col, n, a, u, v, bad)) ++kept;
  }
  uint32_t total = 0;
  int64_t at = off[blockIdx.x] + csr_block_scan(kept, wsum, &total);
  for (int k = 0; k < kCsrPer; ++k) {
    const int64_t a = a0 + k;
    if (a >= nnz) break;
    int32_t u, v;
    if (!csr_keep(row_ptr, col, n, a, u, v, bad)) continue;
    out_src[at] = u;
    out_dst[at] = v;
    out_w[at] = w[a];
    ++at;
  }
}

int64_t csr_tiles(int64_t nnz) { return (nnz + kCsrTile - 1) / kCsrTile; }

hipError_t launch_csr_to_edges(int32_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col, const uint32_t* w,
                               uint32_t* cnt, int64_t* off, uint32_t* err, int32_t* out_src, int32_t* out_dst,
                               uint32_t* out_w, hipStream_t s) {
  const int64_t ntiles = csr_tiles(nnz);
  const int grid_rows = (int)std::min<int64_t>(4096, std::max<int64_t>(1, ((int64_t)n + kCsrBlock - 1) / kCsrBlock));
  k_csr_check_rows<<<grid_rows, kCsrBlock, 0, s>>>(n, nnz, row_ptr, err);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || ntiles == 0) return e;
  if (ntiles > 0x7FFFFFFF) return hipErrorInvalidValue;
  k_csr_count<<<(unsigned)ntiles, kCsrBlock, 0, s>>>(n, nnz, row_ptr, col, cnt, err);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  k_csr_scan<<<1, kCsrBlock, 0, s>>>(ntiles, cnt, off);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  k_csr_scatter<<<(unsigned)ntiles, kCsrBlock, 0, s>>>(n, nnz, row_ptr, col, w, off, out_src, out_dst, out_w);
  return hipGetLastError();
}

}  // namespace mstx
