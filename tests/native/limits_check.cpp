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
  std::printf(fails ? "limits: %d failures\n" : "limits: ok\n", fails);
  return fails ? 1 : 0;
}
