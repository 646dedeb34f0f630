// Test infrastructure (no GPU code): checks a block of rows of a network in
// compressed sparse row form against its cells, and accumulates the
// order-independent pair checksum that the CPU oracle computes over its WSPD
// pairs.  Built with g++ by tests/test_gpu_parity.py; the library never
// links it.
//
// Network layout (the one the library and the oracle share, Sec. 5.3 and
// Alg. 7): nodes 0..n-1 are cells, n the A-diagonal node, n+1 the
// B-diagonal node; row v holds the arcs out of v with strictly increasing
// heads; a cell's arcs go to cells (cost 2 max(|di|, |dj|)) and, when the
// cell holds A mass, last to node n (cost j - i); row n is empty; row n+1
// goes to every cell with B mass (cost j - i), then to node n (cost 0).
#include <cstdint>
#include <cstdlib>

namespace {

// The oracle's pair checksum term of the WSPD pair (u, v, c), u < v.
inline uint64_t pair_mix(uint64_t u, uint64_t v, uint64_t c) {
  uint64_t x = ((u + 1) * 0x9E3779B97F4A7C15ull + (v + 1)) * 0xC2B2AE3D27D4EB4Full + c;
  return x * 0x165667B19E3779F9ull;
}

}  // namespace

extern "C" {

// Rows [r0, r1) of a network with n cells; row_ptr (n + 3 entries) is the
// full pointer array, col / cost hold arcs [a0, a0 + len).  sums[0..1]: the
// checksum (sum, sum of squares) over cell arcs with tail < head taken as
// pairs (tail, head); sums[2..3]: over arcs with tail > head taken as
// (head, tail).  counts[0..1]: the numbers of those arcs.  Returns the
// number of violations found; *first_bad gets the first bad row (or -1).
int64_t csr_check_rows(int64_t n, int64_t r0, int64_t r1, const int64_t* row_ptr, int64_t a0, int64_t len,
                       const uint32_t* col, const int32_t* cost, const int32_t* ci, const int32_t* cj,
                       const int32_t* ca, const int32_t* cb, uint64_t* sums, int64_t* counts, int64_t* first_bad) {
  int64_t bad = 0, first = -1;
  uint64_t s0 = 0, s1 = 0, s2 = 0, s3 = 0;
  int64_t c0 = 0, c1 = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : bad, s0, s1, s2, s3, c0, c1)
  for (int64_t r = r0; r < r1; ++r) {
    const int64_t a = row_ptr[r], e = row_ptr[r + 1];
    bool ok = a <= e && a >= a0 && e <= a0 + len;
    if (ok && r < n) {
      int64_t prev = -1;
      for (int64_t k = a; ok && k < e; ++k) {
        const int64_t h = col[k - a0];
        if (h <= prev) ok = false;
        prev = h;
        if (h < n) {
          const int64_t di = std::llabs((int64_t)ci[r] - ci[h]), dj = std::llabs((int64_t)cj[r] - cj[h]);
          if (cost[k - a0] != 2 * (di > dj ? di : dj) || h == r) ok = false;
          const uint64_t u = (uint64_t)(r < h ? r : h), v = (uint64_t)(r < h ? h : r);
          const uint64_t x = pair_mix(u, v, (uint64_t)(int64_t)cost[k - a0]);
          if (r < h) {
            s0 += x;
            s1 += x * x;
            ++c0;
          } else {
            s2 += x;
            s3 += x * x;
            ++c1;
          }
        } else if (h == n) {
          if (k != e - 1 || ca[r] <= 0 || cost[k - a0] != cj[r] - ci[r]) ok = false;
        } else {
          ok = false;
        }
      }
      if (ok && ca[r] > 0 && (e == a || col[e - 1 - a0] != (uint32_t)n)) ok = false;
    } else if (ok && r == n) {
      ok = a == e;
    } else if (ok && r == n + 1) {
      int64_t k = a;
      for (int64_t c = 0; ok && c < n; ++c)
        if (cb[c] > 0) {
          if (k >= e || col[k - a0] != (uint32_t)c || cost[k - a0] != cj[c] - ci[c]) ok = false;
          ++k;
        }
      ok = ok && k == e - 1 && col[k - a0] == (uint32_t)n && cost[k - a0] == 0;
    } else if (ok) {
      ok = false;  // no such row
    }
    if (!ok) {
      ++bad;
#pragma omp critical
      if (first < 0 || r < first) first = r;
    }
  }
  sums[0] += s0;
  sums[1] += s1;
  sums[2] += s2;
  sums[3] += s3;
  counts[0] += c0;
  counts[1] += c1;
  if (first_bad) *first_bad = first;
  return bad;
}

}  // extern "C"
