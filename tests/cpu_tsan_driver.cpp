// Runs the CPU Boruvka variants of libmstx_cpu on seeded random graphs with
// several thread counts and checks that every variant returns the tree of the
// sequential one.  Built with -fsanitize=thread by tests/test_cpu_baselines.py.
#include <cstdint>
#include <cstdio>
#include <vector>

#include "mstx_cpu.h"

int main() {
  uint64_t s = 0x9E3779B97F4A7C15ull;
  auto next = [&]() {  // xorshift64*
    s ^= s >> 12;
    s ^= s << 25;
    s ^= s >> 27;
    return (s * 0x2545F4914F6CDD1Dull) >> 32;
  };
  int failures = 0;
  for (int gidx = 0; gidx < 3; ++gidx) {
    const int32_t n = 2000 + 700 * gidx;
    const int64_t m = 6 * (int64_t)n;
    std::vector<int32_t> src(m), dst(m);
    std::vector<uint32_t> w(m);
    for (int64_t e = 0; e < m; ++e) {
      // a path keeps it connected; the rest are random pairs with few distinct weights
      src[e] = e < n - 1 ? (int32_t)e : (int32_t)(next() % n);
      dst[e] = e < n - 1 ? (int32_t)(e + 1) : (int32_t)(next() % n);
      w[e] = (uint32_t)(next() % 50);
    }
    std::vector<uint8_t> ref(m), got(m);
    uint64_t ref_total = 0, total = 0;
    const int st0 = mst_cpu_solve(MSTX_CPU_SEQ_COVERED, 1, n, m, src.data(), dst.data(), w.data(), ref.data(),
                                  &ref_total, nullptr);
    for (int variant : {MSTX_CPU_SEQ_PLAIN, MSTX_CPU_PAR_LOCK, MSTX_CPU_PAR_CAS}) {
      for (int threads : {1, 2, 4, 8}) {
        const int st = mst_cpu_solve(variant, threads, n, m, src.data(), dst.data(), w.data(), got.data(), &total,
                                     nullptr);
        if (st != st0 || total != ref_total || got != ref) {
          std::printf("mismatch: graph %d variant %d threads %d status %d/%d\n", gidx, variant, threads, st, st0);
          ++failures;
        }
      }
    }
  }
  std::printf(failures ? "FAILED\n" : "ok\n");
  return failures ? 1 : 0;
}
