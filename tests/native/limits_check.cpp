// Plain C++ check of the host-side work-list limits (built with g++ by
// tests/test_host_limits.py; no GPU).
#include <cstdint>
#include <cstdio>

#include "../../paper_2110_14734_amd/csrc/limits.h"

static int fails = 0;
#define EXPECT(c)                                          \
  do {                                                     \
    if (!(c)) {                                            \
      std::printf("FAILED: %s (line %d)\n", #c, __LINE__); \
      ++fails;                                             \
    }                                                      \
  } while (0)

int main() {
  const int64_t two31 = int64_t(1) << 31;
  EXPECT(w1::worklist_round_fits(0));
  EXPECT(w1::worklist_round_fits(two31 - 1));
  EXPECT(!w1::worklist_round_fits(two31));
  EXPECT(!w1::worklist_round_fits(-1));
  // the largest frontier that fits keeps both packed sums inside 32 bits
  const uint64_t f = (uint64_t)(two31 - 1);
  EXPECT(f <= 0xffffffffull && 2 * f <= 0xffffffffull);
  EXPECT(w1::worklist_items_fit(two31 - 1));
  EXPECT(!w1::worklist_items_fit(two31));
  EXPECT(!w1::worklist_items_fit(int64_t(3) << 33));
  EXPECT(w1::worklist_chunks_fit(12345));
  EXPECT(!w1::worklist_chunks_fit(two31));
  // the last item index of a list that fits is a valid int32
  EXPECT((int64_t)(int32_t)(two31 - 2) == two31 - 2);
  // network row form: the 200k + 200k-point pair (399,980 cells) takes
  // 512-cell buckets and 19-bit heads
  w1::CsrGeometry g = w1::csr_geometry(399980, 399980);
  EXPECT(g.ok && g.RB == 9 && g.DB == 19 && g.NB == 782);
  // a launch group of many small pairs: larger buckets, few head bits
  g = w1::csr_geometry(4000000, 100000);
  EXPECT(g.ok && g.RB == 12 && g.DB == 17 && g.NB <= 1024);
  // heads must be representable: the first count that needs one more bit
  EXPECT(w1::csr_geometry(1, 1).ok && w1::csr_geometry(1, 1).DB == 1);
  EXPECT(w1::csr_geometry(3, 3).DB == 2 && w1::csr_geometry(4, 4).DB == 2 && w1::csr_geometry(5, 5).DB == 3);
  // beyond 2^22 cells in one launch group there would be more than 1024 buckets
  EXPECT(w1::csr_geometry(int64_t(1) << 22, 1000).ok);
  EXPECT(!w1::csr_geometry((int64_t(1) << 22) + 1, 1000).ok);
  // a 2.8M-cell pair needs 22 head bits and 4096-cell buckets: 34 bits
  EXPECT(!w1::csr_geometry(2800000, 2800000).ok);
  // every tail within a bucket and every head fit the 32-bit entry
  const int64_t sizes[] = {1, 2, 511, 512, 513, 400000, 1000000, 4194304};
  for (int64_t n : sizes) {
    const w1::CsrGeometry q = w1::csr_geometry(n, n);
    if (!q.ok) continue;
    EXPECT(q.NB * (int64_t(1) << q.RB) >= n && (q.NB - 1) * (int64_t(1) << q.RB) < n);
    EXPECT((int64_t(1) << q.DB) >= n && q.RB + q.DB <= 32);
  }
  std::printf(fails ? "limits: %d failures\n" : "limits: ok\n", fails);
  return fails ? 1 : 0;
}
