// a5: the sparse transshipment network in compressed sparse row form.
//
// The network simplex reads the network as a static CSR graph: the arcs
// sorted by tail, ties by head (Appendix, network representation).  The
// paper sorts its arc list with a parallel merge sort; here the sort is a
// two-level partition followed by a per-row bitmap sort, which moves each
// arc a fixed number of times and never sorts more than one row at once:
//
//   1. bucket histogram: each arc u -> v of a WSPD pair record (both
//      orientations) counts towards the bucket of its tail, a bucket being
//      2^RB consecutive global cells (taken by the WSPD emit pass as it
//      writes the records);
//   2. bucket scatter: arcs are written bucket-major as 32-bit entries
//      (tail within the bucket << DB | head), staged in LDS so each block
//      writes one contiguous run per bucket;
//   3. row histogram, per bucket: the out-degree of every cell;
//   4. row scatter, per bucket: each row's heads are written to the row's
//      final place (order within the row still arbitrary);
//   5. row sort: one block per row sets one bit per head in an LDS bitmap
//      over the pair's cells and reads the bits back in order through
//      per-wave LDS staging, writing the heads and their costs (2 max(|di|,
//      |dj|) from the cell coordinates) coalesced, and the row's arc to the
//      A-diagonal node;
//   6. the B-diagonal node's row: its arcs to the cells with B mass, in cell
//      order, then to the A-diagonal node; and the supplies.
//
// Heads are distinct within a row (a repeated arc would mean a cell pair
// covered by two WSPD pairs), so the bitmap loses nothing and the result is
// the unique sorted order, independent of the arbitrary orders before it.
//
// Row numbering: the rows of diagram pair p are cell_start[p] + 2p + r for
// r in [0, n_p + 2): its cells, then its A-diagonal node (no out-arcs), then
// its B-diagonal node -- the layout of the supply array.  Heads are local
// node ids of the pair (cells 0..n_p-1, A-diagonal n_p, B-diagonal n_p + 1).
#include "common.h"
#include "kernels.h"

namespace w1 {

namespace {

constexpr int CB = 512;        // threads per block of the partition passes
// Tile sizes of the partition passes.  Each is one tile per block with three
// barriers, so occupancy hides more latency than longer output runs save:
// on the 200k + 200k pair (782 buckets) the bucket scatter took 12.9 ms with
// 8 records per thread, 11.7 ms with 4 (2: 14.3 ms); the row scatter 14.7 ms
// with 16 entries per thread, 11.1 ms with 8 (4: 13.8 ms).  The row
// histogram's cost per tile is one atomic per row, so it takes large tiles.
constexpr int PPT = 4;         // pair records per thread in the bucket scatter
constexpr int PTILE = CB * PPT;
constexpr int HIST_EPT = 64;   // entries per thread in the row histogram
// The bucket cursors sit one per 128-byte line: every tile of the bucket
// scatter reserves a run in most buckets, and cursors sharing a line
// serialise those atomics (with 2 records per thread, 17.4 -> 14.3 ms).
constexpr int BCUR_STRIDE = 16;
constexpr int SORT_B = 512;    // threads per block of the row sort
constexpr int SORT_WAVES = SORT_B / WAVE;
constexpr int SORT_STAGE = 512;  // staged heads per wave of the row sort
constexpr int WIN_WORDS = 24576;  // largest bitmap window (96 KiB; with the staging 112 KiB of LDS)
constexpr int SORT_MAXG = WIN_WORDS / WAVE;  // groups of 64 words in a window
constexpr int SORT_FILL = 4;                 // head loads per thread in flight in the row sort
constexpr int SORT_TASKS = 64;               // runs of groups per row window, taken by the waves in turn
constexpr uint32_t SORT_GROUP_W = 32;        // weight of visiting a non-empty group, in heads
constexpr int SORT_DENSE_BATCH = 8;          // cell-coordinate loads in flight per lane, dense groups

// Last p in [0, K) with rstart[p] <= x (the pair holding record x: pairs
// without records share their start with the next pair, which wins).
__device__ inline int64_t pair_of(const uint64_t* __restrict__ rstart, int64_t K, uint64_t x) {
  int64_t lo = 0, hi = K;
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (rstart[mid] <= x) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Diagram pair of every record of a tile: the pair of the first and of the
// last record, found once per block; records in between search only that
// range (almost always one pair).
struct TilePairs {
  int64_t p0, p1;
};
__device__ inline TilePairs tile_pairs(const uint64_t* rstart, int64_t K, uint64_t x0, uint64_t x1) {
  __shared__ int64_t s_p[2];
  if (threadIdx.x == 0) {
    s_p[0] = pair_of(rstart, K, x0);
    s_p[1] = pair_of(rstart, K, x1 - 1);
  }
  __syncthreads();
  return TilePairs{s_p[0], s_p[1]};
}
__device__ inline int64_t record_pair(const TilePairs& tp, const uint64_t* rstart, uint64_t x) {
  if (tp.p0 == tp.p1) return tp.p0;
  int64_t lo = tp.p0, hi = tp.p1 + 1;
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (rstart[mid] <= x) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Exclusive scan of n LDS counters in place (block of CB threads, each
// owning a contiguous run); returns nothing, s_tmp needs CB / WAVE slots.
__device__ inline void lds_excl_scan(uint32_t* cnt, int n, uint32_t* s_tmp) {
  const int per = (n + CB - 1) / CB;
  const int a = threadIdx.x * per, b = min(n, a + per);
  uint32_t sum = 0;
  for (int i = a; i < b; ++i) sum += cnt[i];
  // wave inclusive scan of the run sums
  const int lane = lane_id(), wave = threadIdx.x / WAVE;
  uint32_t inc = sum;
#pragma unroll
  for (int d = 1; d < WAVE; d <<= 1) {
    const uint32_t o = __shfl_up(inc, d);
    if (lane >= d) inc += o;
  }
  if (lane == WAVE - 1) s_tmp[wave] = inc;
  __syncthreads();
  uint32_t pre = inc - sum;
  for (int w = 0; w < wave; ++w) pre += s_tmp[w];
  for (int i = a; i < b; ++i) {
    const uint32_t c = cnt[i];
    cnt[i] = pre;
    pre += c;
  }
  __syncthreads();
}

// ------------------------------------------------------ arcs of a record --
// Arcs of pair record x (rw words per record, u and v first): tail cell
// (global) and entry.
__device__ inline void record_arcs(const uint32_t* __restrict__ rec, uint64_t x, uint32_t rw, int64_t cs, int RB,
                                   int DB, uint32_t& b0, uint32_t& e0, uint32_t& b1, uint32_t& e1) {
  uint32_t u, v;
  if (rw == 2) {  // one 8-byte load
    const uint2 r = ((const uint2*)rec)[x];
    u = r.x;
    v = r.y;
  } else {
    u = rec[rw * x];
    v = rec[rw * x + 1];
  }
  const uint64_t gu = (uint64_t)cs + u, gv = (uint64_t)cs + v;
  const uint32_t m = (1u << RB) - 1u;
  b0 = (uint32_t)(gu >> RB);
  e0 = (((uint32_t)gu & m) << DB) | v;
  b1 = (uint32_t)(gv >> RB);
  e1 = (((uint32_t)gv & m) << DB) | u;
}

// ------------------------------------------------------- 2. bucket scatter --
__global__ void __launch_bounds__(CB) k_bucket_scatter(const uint32_t* __restrict__ rec, uint64_t P,
                                                       const uint64_t* __restrict__ rstart, int64_t K,
                                                       const int64_t* __restrict__ cell_start, int RB, int DB, int NB,
                                                       const uint64_t* __restrict__ bstart,
                                                       unsigned long long* __restrict__ bcur,
                                                       uint32_t* __restrict__ out,
                                                       const uint32_t* __restrict__ blk_fill,
                                                       const uint32_t* __restrict__ blk_pair, uint32_t blk_recs,
                                                       uint32_t rw, int cstride) {
  extern __shared__ uint32_t s_mem[];
  uint32_t* s_cnt = s_mem;                         // NB: counts, then prefixes
  int64_t* s_gofs = (int64_t*)(s_mem + ((NB + 1) & ~1));  // NB: global base - prefix
  uint32_t* s_ent = (uint32_t*)(s_gofs + NB);      // 2 PTILE staged entries
  uint16_t* s_bkt = (uint16_t*)(s_ent + 2 * PTILE);  // 2 PTILE bucket ids
  __shared__ uint32_t s_tmp[CB / WAVE];
  // a tile: PTILE consecutive records of rw words ((u, v) or (u, v, cost)),
  // or one block of the blocked emission (records (u, v); its fill and
  // diagram pair given)
  const uint64_t x0 = (uint64_t)blockIdx.x * (blk_fill ? blk_recs : (uint32_t)PTILE);
  const uint64_t x1 = blk_fill ? x0 + blk_fill[blockIdx.x] : min(P, x0 + PTILE);
  for (int b = threadIdx.x; b < NB; b += CB) s_cnt[b] = 0;
  __syncthreads();  // every counter is zero before any thread counts
  const TilePairs tp = blk_fill ? TilePairs{(int64_t)blk_pair[blockIdx.x], (int64_t)blk_pair[blockIdx.x]}
                                : tile_pairs(rstart, K, x0, x1);
  uint32_t eb[2 * PPT], ee[2 * PPT], er[2 * PPT];
  int n = 0;
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const uint64_t x = x0 + (uint64_t)k * CB + threadIdx.x;
    if (x < x1) {
      const int64_t cs = cell_start[record_pair(tp, rstart, x)];
      record_arcs(rec, x, rw, cs, RB, DB, eb[2 * k], ee[2 * k], eb[2 * k + 1], ee[2 * k + 1]);
      er[2 * k] = atomicAdd(&s_cnt[eb[2 * k]], 1u);
      er[2 * k + 1] = atomicAdd(&s_cnt[eb[2 * k + 1]], 1u);
      n = 2 * k + 2;
    }
  }
  __syncthreads();
  // reserve each bucket's run in the global bucket, then turn counts into
  // block-local prefixes
  for (int b = threadIdx.x; b < NB; b += CB) {
    const uint32_t c = s_cnt[b];
    s_gofs[b] = c ? (int64_t)(bstart[b] + atomicAdd(&bcur[(int64_t)b * cstride], (unsigned long long)c)) : 0;
  }
  __syncthreads();
  lds_excl_scan(s_cnt, NB, s_tmp);
  for (int b = threadIdx.x; b < NB; b += CB) s_gofs[b] -= (int64_t)s_cnt[b];
#pragma unroll
  for (int k = 0; k < 2 * PPT; ++k) {
    if (k < n) {
      const uint32_t pos = s_cnt[eb[k]] + er[k];
      s_ent[pos] = ee[k];
      s_bkt[pos] = (uint16_t)eb[k];
    }
  }
  __syncthreads();
  const uint32_t tot = (uint32_t)(2 * (x1 - x0));
  for (uint32_t i = threadIdx.x; i < tot; i += CB) out[s_gofs[s_bkt[i]] + (int64_t)i] = s_ent[i];
}

// ------------------------------------------------------ 3. / 4. row passes --
// Tile t of the bucket-major entries: bucket b = last with tfirst[b] <= t.
struct BTile {
  int64_t b, a, e;  // bucket, entry range [a, e)
};
__device__ inline BTile bucket_tile(const int64_t* __restrict__ tfirst, int NB, const uint64_t* __restrict__ bstart,
                                    int64_t t, int etile) {
  __shared__ int64_t s_t[3];
  if (threadIdx.x == 0) {
    int64_t lo = 0, hi = NB;
    while (hi - lo > 1) {
      const int64_t mid = (lo + hi) >> 1;
      if (tfirst[mid] <= t) lo = mid;
      else hi = mid;
    }
    const int64_t a = (int64_t)bstart[lo] + (t - tfirst[lo]) * etile;
    s_t[0] = lo;
    s_t[1] = a;
    s_t[2] = min((int64_t)bstart[lo + 1], a + etile);
  }
  __syncthreads();
  return BTile{s_t[0], s_t[1], s_t[2]};
}

__global__ void __launch_bounds__(CB) k_row_hist(const uint32_t* __restrict__ ent, const int64_t* __restrict__ tfirst,
                                                 int NB, const uint64_t* __restrict__ bstart, int RB, int DB,
                                                 int64_t N, int etile, uint32_t* __restrict__ rowcnt) {
  extern __shared__ uint32_t s_hist[];
  const int R = 1 << RB;
  for (int r = threadIdx.x; r < R; r += CB) s_hist[r] = 0;
  const BTile bt = bucket_tile(tfirst, NB, bstart, blockIdx.x, etile);
  for (int64_t i = bt.a + threadIdx.x; i < bt.e; i += CB) atomicAdd(&s_hist[ent[i] >> DB], 1u);
  __syncthreads();
  const int64_t g0 = bt.b << RB;
  for (int r = threadIdx.x; r < R; r += CB)
    if (s_hist[r] && g0 + r < N) atomicAdd(&rowcnt[g0 + r], s_hist[r]);
}

// EPT entries per thread: the tile of CB * EPT entries and the 2^RB row
// counters share the LDS (EPT = 8 up to 2^11 rows per bucket).
template <int EPT>
__global__ void __launch_bounds__(CB) k_row_scatter(const uint32_t* __restrict__ ent, const int64_t* __restrict__ tfirst,
                                                    int NB, const uint64_t* __restrict__ bstart, int RB, int DB,
                                                    int64_t N, const uint32_t* __restrict__ cpair,
                                                    const uint64_t* __restrict__ off, uint32_t* __restrict__ rowcur,
                                                    uint32_t* __restrict__ heads) {
  extern __shared__ uint32_t s_mem[];
  const int R = 1 << RB;
  uint32_t* s_cnt = s_mem;
  int64_t* s_gofs = (int64_t*)(s_mem + R);
  uint32_t* s_ent = (uint32_t*)(s_gofs + R);
  uint16_t* s_row = (uint16_t*)(s_ent + CB * EPT);
  __shared__ uint32_t s_tmp[CB / WAVE];
  for (int r = threadIdx.x; r < R; r += CB) s_cnt[r] = 0;
  const BTile bt = bucket_tile(tfirst, NB, bstart, blockIdx.x, CB * EPT);
  uint32_t ev[EPT], rk[EPT];
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const int64_t i = bt.a + (int64_t)k * CB + threadIdx.x;
    if (i < bt.e) {
      ev[k] = ent[i];
      rk[k] = atomicAdd(&s_cnt[ev[k] >> DB], 1u);
    }
  }
  __syncthreads();
  const int64_t g0 = bt.b << RB;
  for (int r = threadIdx.x; r < R; r += CB) {
    const uint32_t c = s_cnt[r];
    int64_t base = 0;
    if (c) {
      const int64_t g = g0 + r;
      base = (int64_t)off[g + 2 * (int64_t)cpair[g]] + (int64_t)atomicAdd(&rowcur[g], c);
    }
    s_gofs[r] = base;
  }
  __syncthreads();
  lds_excl_scan(s_cnt, R, s_tmp);
  for (int r = threadIdx.x; r < R; r += CB) s_gofs[r] -= (int64_t)s_cnt[r];
  const uint32_t hmask = (1u << DB) - 1u;
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const int64_t i = bt.a + (int64_t)k * CB + threadIdx.x;
    if (i < bt.e) {
      const uint32_t r = ev[k] >> DB;
      const uint32_t pos = s_cnt[r] + rk[k];
      s_ent[pos] = ev[k] & hmask;
      s_row[pos] = (uint16_t)r;
    }
  }
  __syncthreads();
  const int tot = (int)(bt.e - bt.a);
  for (int i = threadIdx.x; i < tot; i += CB) heads[s_gofs[s_row[i]] + i] = s_ent[i];
}

// ------------------------------------------------------------ 5. row sort --
// Exclusive prefix over the wave's lanes of v < 2^NB, and the wave total,
// from NB ballots (one per bit plane) and lane-mask counts: no cross-lane
// data movement, so no memory round trip.
template <int NB>
__device__ inline uint32_t wave_excl_prefix(uint32_t v, uint32_t& total) {
  uint32_t ex = 0, tot = 0;
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const uint64_t m = __ballot((v >> b) & 1u);
    ex += __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u)) << b;
    tot += (uint32_t)__popcll(m) << b;
  }
  total = tot;
  return ex;
}

// Exclusive prefix of small counts: one ballot per unit of the largest
// count (sum over j of the lanes below with v > j), cheaper than bit planes
// when the counts are mostly 0 or 1.
__device__ inline uint32_t wave_excl_prefix_small(uint32_t v) {
  uint32_t ex = 0;
  for (uint32_t j = 0;; ++j) {
    const uint64_t m = __ballot(v > j);
    if (m == 0) break;
    ex += __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
  }
  return ex;
}

// Arc costs.  L-infinity (int32, units of g/2): 2 max(|di|, |dj|) between
// cells, j - i to the diagonal.  Euclidean (int64, units of g 2^-K): the
// distances of the cell centres rounded up, ceil(sqrt(di^2 + dj^2) 2^K) and
// ceil((j - i) R 2^K), each from IEEE double operations in this order (the
// integer sum converted to double, correctly rounded square root, exact
// scaling by 2^K).
template <bool L2>
struct ArcCost;

template <>
struct ArcCost<false> {
  typedef int32_t T;
  __device__ static T cell(int2 a, int2 b, int) { return 2 * max(abs(a.x - b.x), abs(a.y - b.y)); }
  __device__ static T diag(int2 a, int) { return a.y - a.x; }
};

template <>
struct ArcCost<true> {
  typedef int64_t T;
  __device__ static T cell(int2 a, int2 b, int K) {
    const int64_t di = (int64_t)a.x - b.x, dj = (int64_t)a.y - b.y;
    return (int64_t)ceil(ldexp(sqrt((double)(di * di + dj * dj)), K));
  }
  __device__ static T diag(int2 a, int K) {
    return (int64_t)ceil(ldexp((double)(a.y - a.x) * 0x1.6a09e667f3bcdp-1, K));
  }
};

// Writes a wave's staged heads (in order) as arcs k0, k0 + 1, ... of the row
// of cell `me`: head and cost.  Four heads per lane are in flight at once, so
// their cell-coordinate gathers overlap.
template <bool L2>
__device__ inline void flush_staged(const uint32_t* st, uint32_t n, int64_t k0, int2 me, const int2* __restrict__ cij,
                                    int64_t cs, int K, uint32_t* __restrict__ col,
                                    typename ArcCost<L2>::T* __restrict__ cost) {
  const uint32_t lane = (uint32_t)lane_id();
  for (uint32_t x = lane; x < n; x += 4 * WAVE) {
    uint32_t d[4];
    int2 o[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) d[u] = x + u * WAVE < n ? st[x + u * WAVE] : 0u;
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (x + u * WAVE < n) o[u] = cij[cs + d[u]];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (x + u * WAVE < n) {
        const int64_t k = k0 + x + u * WAVE;
        col[k] = d[u];
        cost[k] = ArcCost<L2>::cell(me, o[u], K);
      }
  }
}

// Persistent blocks, each sorting rows g = blockIdx.x, + gridDim.x, ...
// heads: a row's heads in arbitrary order (rowcnt[g] of them at off[row]);
// col / cost: the sorted row.  Per row (and per window of `win_words`
// bitmap words over the pair's cells):
//   1. each head sets its bit in an LDS bitmap (the first SORT_FILL * SORT_B
//      heads were loaded while the previous row was being written); the set
//      bits are then counted per group of 64 words by popcount;
//   2. the group counts are scanned, and the groups are cut into SORT_TASKS
//      runs of about equal weight, a group weighing its heads plus
//      SORT_GROUP_W (the fixed cost of visiting it): a row's heads crowd
//      around its own cell, so equal runs of words would be very uneven;
//   3. the waves take the runs in turn as they finish the previous one, read
//      the run's non-empty groups in order (clearing the words behind them,
//      so the bitmap is zero again for the next row), expand the set bits
//      into their LDS staging areas and write the staged heads with their
//      costs coalesced; a group denser than the staging area is written
//      straight from its words, 64 consecutive cells per step.
// At most 128 VGPRs (4 waves per SIMD), so that two blocks share a compute
// unit: the Euclidean variant compiled to 129 on its own, which halved the
// blocks per compute unit and took its pass from 36.6 to 55.8 ms.
template <bool L2>
__global__ void __launch_bounds__(SORT_B) __attribute__((amdgpu_waves_per_eu(4))) k_row_sort(const uint32_t* __restrict__ cpair,
                                                     const int64_t* __restrict__ cell_start,
                                                     const int32_t* __restrict__ ncells, const int2* __restrict__ cij,
                                                     const int32_t* __restrict__ ca, const uint32_t* __restrict__ rowcnt,
                                                     const uint64_t* __restrict__ off,
                                                     const uint32_t* __restrict__ heads, int64_t N, int win_words,
                                                     const int32_t* __restrict__ costK, uint32_t* __restrict__ col,
                                                     typename ArcCost<L2>::T* __restrict__ cost,
                                                     unsigned long long* __restrict__ rowq) {
  extern __shared__ uint32_t s_mem[];
  __shared__ int64_t s_nextg;                 // the block's next row, from the row queue
  __shared__ uint32_t s_gpre[SORT_MAXG + 1];  // heads per group, then their exclusive prefix
  __shared__ uint32_t s_wpre[SORT_MAXG];      // exclusive prefix of the group weights
  __shared__ int s_task[SORT_TASKS + 1];      // first group of each run
  __shared__ int s_next;                      // next run to take
  const int lane = lane_id(), wave = threadIdx.x / WAVE;
  uint32_t* s_bm = s_mem;
  uint32_t* s_st = s_mem + win_words + wave * SORT_STAGE;
  for (int i = threadIdx.x; i < win_words; i += SORT_B) s_bm[i] = 0;
  // the first SORT_FILL * SORT_B heads of a row, loaded ahead (~0: none)
  uint32_t pre[SORT_FILL];
  auto load_ahead = [&](int64_t r) {
#pragma unroll
    for (int u = 0; u < SORT_FILL; ++u) pre[u] = ~0u;
    if (r >= N) return;
    const uint32_t n = rowcnt[r];
    const int64_t st = (int64_t)off[r + 2 * (int64_t)cpair[r]];
#pragma unroll
    for (int u = 0; u < SORT_FILL; ++u)
      if (threadIdx.x + u * SORT_B < n) pre[u] = heads[st + threadIdx.x + u * SORT_B];
  };
  load_ahead(blockIdx.x);
  // rows: blockIdx.x first, then from a queue (rows gridDim.x, gridDim.x + 1,
  // ... in the order blocks ask), so that blocks with shorter rows take more
  // of them; thread 0 takes the next row during the fill
  int64_t nextg = N;
  for (int64_t g = blockIdx.x; g < N; g = nextg) {
    const uint32_t p = cpair[g];
    const int64_t cs = cell_start[p];
    const uint32_t np = (uint32_t)ncells[p];
    const int64_t start = (int64_t)off[g + 2 * (int64_t)p];
    const uint32_t cnt = rowcnt[g];
    const int2 me = cij[g];
    const int K = L2 ? costK[p] : 0;
    uint32_t written = 0;  // heads written by earlier windows (block-uniform)
    bool ahead = true;     // pre[] still holds this row's first heads
    for (uint32_t w0 = 0; cnt > 0 && w0 < np; w0 += 32u * (uint32_t)win_words) {
      const uint32_t nbits = min(np - w0, 32u * (uint32_t)win_words);
      const int nw = (int)((nbits + 31) / 32);
      const int ng = (nw + WAVE - 1) / WAVE;
      for (int q = threadIdx.x; q <= ng; q += SORT_B) s_gpre[q] = 0;
      __syncthreads();  // also orders the previous row's last reads before this row's bits
      if (ahead && threadIdx.x == 0) s_nextg = (int64_t)gridDim.x + (int64_t)atomicAdd(rowq, 1ull);
      for (uint32_t i0 = threadIdx.x; i0 < cnt; i0 += SORT_FILL * SORT_B) {
        uint32_t h[SORT_FILL];  // all loads in flight before the first bit is set
        if (i0 == threadIdx.x && w0 == 0) {
#pragma unroll
          for (int u = 0; u < SORT_FILL; ++u) h[u] = pre[u];
        } else {
#pragma unroll
          for (int u = 0; u < SORT_FILL; ++u)
            h[u] = i0 + u * SORT_B < cnt ? heads[start + i0 + u * SORT_B] - w0 : ~0u;
        }
#pragma unroll
        for (int u = 0; u < SORT_FILL; ++u)
          if (h[u] < nbits) atomicOr(&s_bm[h[u] >> 5], 1u << (h[u] & 31));
      }
      __syncthreads();
      // heads per group: each thread counts eight words by popcount and adds
      // them with one LDS atomic (an atomic per head on the group counters
      // serialised the dense groups' heads)
      for (int i0 = threadIdx.x * 8; i0 < nw; i0 += SORT_B * 8) {
        uint32_t v = 0;
        if (i0 + 8 <= nw) {
          const uint4 a = *(const uint4*)(s_bm + i0), b = *(const uint4*)(s_bm + i0 + 4);
          v = __popc(a.x) + __popc(a.y) + __popc(a.z) + __popc(a.w) + __popc(b.x) + __popc(b.y) + __popc(b.z) +
              __popc(b.w);
        } else {
          for (int k = i0; k < nw; ++k) v += __popc(s_bm[k]);
        }
        if (v) atomicAdd(&s_gpre[i0 >> 6], v);
      }
      __syncthreads();
      if (ahead) {  // the next row's first heads arrive while this one is written
        nextg = s_nextg;
        load_ahead(nextg);
        ahead = false;
      }
      if (wave == 0) {  // exclusive scans of the heads and weights per group, then the runs
        uint32_t carry = 0, wcarry = 0;
        for (int c0 = 0; c0 < ng; c0 += WAVE) {
          const int q = c0 + lane;
          const uint32_t v = q < ng ? s_gpre[q] : 0u;
          uint32_t t;
          const uint32_t ex = wave_excl_prefix<12>(v, t);
          const uint64_t ne = __ballot(v > 0);
          const uint32_t nex = __builtin_amdgcn_mbcnt_hi((uint32_t)(ne >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)ne, 0u));
          if (q < ng) {
            s_gpre[q] = carry + ex;
            s_wpre[q] = wcarry + ex + SORT_GROUP_W * nex;
          }
          carry += t;
          wcarry += t + SORT_GROUP_W * (uint32_t)__popcll(ne);
        }
        if (lane == 0) {
          s_gpre[ng] = carry;
          s_task[SORT_TASKS] = ng;
          s_next = 0;
        }
        // run `lane` starts at the first group whose weight prefix reaches
        // lane / SORT_TASKS of the total
        const uint32_t target = (uint32_t)(((uint64_t)wcarry * (uint32_t)lane) / SORT_TASKS);
        int lo = 0, hi = ng;
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (s_wpre[mid] >= target) hi = mid;
          else lo = mid + 1;
        }
        s_task[lane] = lo;
      }
      __syncthreads();
      for (;;) {
        int t = 0;
        if (lane == 0) t = atomicAdd(&s_next, 1);
        t = __shfl(t, 0);
        if (t >= SORT_TASKS) break;
        const int qa = s_task[t], qb = s_task[t + 1];
        if (qa >= qb) continue;
        int64_t k0 = start + written + s_gpre[qa];  // next arc of this run
        uint32_t staged = 0;                         // wave-uniform
        for (int q = qa; q < qb; ++q) {
          const uint32_t tot = s_gpre[q + 1] - s_gpre[q];
          if (tot == 0) continue;
          const int i = q * WAVE + lane;
          const uint32_t word = i < nw ? s_bm[i] : 0u;
          if (staged + tot > SORT_STAGE) {
            __builtin_amdgcn_wave_barrier();
            flush_staged<L2>(s_st, staged, k0, me, cij, cs, K, col, cost);
            k0 += staged;
            staged = 0;
            __builtin_amdgcn_wave_barrier();
          }
          if (tot <= SORT_STAGE) {  // each lane expands its word into the staging area
            uint32_t bits = word, pos = staged + wave_excl_prefix_small((uint32_t)__popc(word));
            while (bits) {
              const int bit = __ffs(bits) - 1;
              bits &= bits - 1;
              s_st[pos++] = w0 + (uint32_t)i * 32u + (uint32_t)bit;
            }
            staged += tot;
          } else {
            // denser than the staging area: written straight from the words,
            // 64 consecutive cells per step (lane l takes cell 64 t + l of
            // the group): a set bit goes to the run's cursor plus the set
            // bits before it, and the cells' coordinates come in coalesced
            uint32_t wt;
            const uint32_t wpre = wave_excl_prefix<6>((uint32_t)__popc(word), wt);
            const uint32_t c0 = w0 + (uint32_t)q * (uint32_t)(WAVE * 32);
            const uint32_t bit = (uint32_t)lane & 31u;
            for (int t0 = 0; t0 < 32; t0 += SORT_DENSE_BATCH) {
              int2 o[SORT_DENSE_BATCH];
#pragma unroll
              for (int u = 0; u < SORT_DENSE_BATCH; ++u) {
                const uint32_t cell = c0 + (uint32_t)(t0 + u) * WAVE + (uint32_t)lane;
                o[u] = cell < np ? cij[cs + cell] : make_int2(0, 0);
              }
#pragma unroll
              for (int u = 0; u < SORT_DENSE_BATCH; ++u) {
                const int wi = 2 * (t0 + u) + (lane >> 5);  // the word holding this lane's cell
                const uint32_t wv = (uint32_t)__shfl((int)word, wi);
                const uint32_t wp = (uint32_t)__shfl((int)wpre, wi);
                if ((wv >> bit) & 1u) {
                  const int64_t k = k0 + wp + (uint32_t)__popc(wv & ((1u << bit) - 1u));
                  col[k] = c0 + (uint32_t)(t0 + u) * WAVE + (uint32_t)lane;
                  cost[k] = ArcCost<L2>::cell(me, o[u], K);
                }
              }
            }
            k0 += tot;
          }
          if (i < nw) s_bm[i] = 0;  // zero again for the next row
        }
        __builtin_amdgcn_wave_barrier();
        flush_staged<L2>(s_st, staged, k0, me, cij, cs, K, col, cost);
        __builtin_amdgcn_wave_barrier();
      }
      written += s_gpre[ng];
      __syncthreads();
    }
    if (ahead) {  // a row without heads
      __syncthreads();  // every thread has read the previous row's s_nextg
      if (threadIdx.x == 0) s_nextg = (int64_t)gridDim.x + (int64_t)atomicAdd(rowq, 1ull);
      __syncthreads();
      nextg = s_nextg;
      load_ahead(nextg);
    }
    if (threadIdx.x == 0 && ca[g] > 0) {  // arc to the A-diagonal node, last in the row
      col[start + cnt] = np;
      cost[start + cnt] = ArcCost<L2>::diag(me, K);
    }
  }
}

// ----------------------------------------------------- degrees and diagonal --
// Out-degree of every row: a cell has its WSPD arcs plus one arc to the
// A-diagonal node when it holds A mass; the A-diagonal node has none; the
// B-diagonal node has one arc per cell with B mass plus one to the
// A-diagonal node.  bpos: exclusive scan of (cb > 0) over all cells.
__global__ void k_row_deg(const uint32_t* __restrict__ cpair, const int64_t* __restrict__ cell_start,
                          const int32_t* __restrict__ ncells, const int32_t* __restrict__ ca,
                          const int32_t* __restrict__ cb, const uint32_t* __restrict__ rowcnt,
                          const uint32_t* __restrict__ bpos, int64_t N, uint64_t* __restrict__ deg) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N) return;
  const uint32_t p = cpair[g];
  const int64_t cs = cell_start[p];
  const int64_t row = g + 2 * (int64_t)p;
  deg[row] = (uint64_t)rowcnt[g] + (ca[g] > 0 ? 1u : 0u);
  if (g - cs == ncells[p] - 1) {
    deg[row + 1] = 0;
    deg[row + 2] = (uint64_t)(bpos[g] + (cb[g] > 0 ? 1u : 0u) - bpos[cs]) + 1u;
  }
}

__global__ void k_bflags(const int32_t* __restrict__ cb, int64_t N, uint32_t* __restrict__ flag) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < N) flag[g] = cb[g] > 0 ? 1u : 0u;
}

// The B-diagonal row and the supplies (cell: A mass minus B mass; A-diagonal
// node: minus the A mass; B-diagonal node: the B mass).
template <bool L2>
__global__ void k_bdiag_rows(const uint32_t* __restrict__ cpair, const int64_t* __restrict__ cell_start,
                             const int32_t* __restrict__ ncells, const int2* __restrict__ cij,
                             const int32_t* __restrict__ ca, const int32_t* __restrict__ cb,
                             const uint32_t* __restrict__ bpos, const uint64_t* __restrict__ off, PairArrays P,
                             int64_t N, const int32_t* __restrict__ costK, uint32_t* __restrict__ col,
                             typename ArcCost<L2>::T* __restrict__ cost, int64_t* __restrict__ supply) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N) return;
  const uint32_t p = cpair[g];
  const int64_t cs = cell_start[p];
  const uint32_t np = (uint32_t)ncells[p];
  const uint32_t local = (uint32_t)(g - cs);
  const int64_t rb = cs + 2 * (int64_t)p + np + 1;  // the B-diagonal row
  const int64_t at = (int64_t)off[rb] + (bpos[g] - bpos[cs]);
  const int2 v = cij[g];
  if (cb[g] > 0) {
    col[at] = local;
    cost[at] = ArcCost<L2>::diag(v, L2 ? costK[p] : 0);
  }
  const int64_t sb = cs + 2 * (int64_t)p;
  supply[sb + local] = (int64_t)ca[g] - (int64_t)cb[g];
  if (local == np - 1) {
    const int64_t last = at + (cb[g] > 0 ? 1 : 0);
    col[last] = np;
    cost[last] = 0;
    supply[sb + np] = -P.nA[p];
    supply[sb + np + 1] = P.nB[p];
  }
}

// Row pointers local to each diagram pair: the n_p + 3 pointers of pair p
// start at cell_start[p] + 3p and count from its first arc.
__global__ void k_local_rowptr(const uint32_t* __restrict__ cpair, const int64_t* __restrict__ cell_start,
                               const int32_t* __restrict__ ncells, const uint64_t* __restrict__ off, int64_t N,
                               int64_t* __restrict__ rp) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N) return;
  const uint32_t p = cpair[g];
  const int64_t cs = cell_start[p];
  const int64_t r0 = cs + 2 * (int64_t)p, local = g - cs;
  const int64_t base = (int64_t)off[r0];
  int64_t* out = rp + cs + 3 * (int64_t)p;
  out[local] = (int64_t)off[r0 + local] - base;
  if (local == ncells[p] - 1)
    for (int r = 1; r <= 3; ++r) out[local + r] = (int64_t)off[r0 + local + r] - base;
}

__global__ void k_pair_arcs(const int64_t* __restrict__ cell_start, const uint64_t* __restrict__ off, int64_t K,
                            int64_t nrows, uint64_t* __restrict__ out) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < K) out[p] = off[cell_start[p] + 2 * p];
  else if (p == K) out[K] = off[nrows];
}

inline unsigned blocks(int64_t n, int bs = 256) { return (unsigned)(n > 0 ? ceil_div(n, bs) : 1); }

}  // namespace

int csr_bucket_stride() { return BCUR_STRIDE; }
size_t csr_bucket_scatter_lds(int NB) {
  return (size_t)((NB + 1) & ~1) * 4 + (size_t)NB * 8 + (size_t)2 * PTILE * (4 + 2);
}
int csr_entries_per_thread(int RB) { return RB <= 11 ? 8 : 4; }
size_t csr_row_scatter_lds(int RB) {
  return (size_t)(1 << RB) * 12 + (size_t)CB * csr_entries_per_thread(RB) * (4 + 2);
}
int64_t csr_entry_tile(int RB) { return (int64_t)CB * csr_entries_per_thread(RB); }
int64_t csr_hist_tile(int) { return (int64_t)CB * HIST_EPT; }

int csr_tile_records() { return PTILE; }
void launch_csr_bucket_scatter(const uint32_t* rec, int rec_words, uint64_t P, const uint64_t* rstart, int64_t K,
                               const int64_t* cell_start, int RB, int DB, int NB, const uint64_t* bstart,
                               uint64_t* bcur, uint32_t* out, const uint32_t* blk_fill, const uint32_t* blk_pair,
                               uint32_t blk_recs, uint32_t nblocks, hipStream_t st) {
  if (P == 0 || (rec_words != 2 && rec_words != 3)) return;
  // blocked records: one tile per block, whose records must fit a tile
  const int ptile = csr_tile_records();
  if (blk_fill && (blk_recs == 0 || blk_recs > (uint32_t)ptile || nblocks == 0)) return;
  const int64_t tiles = blk_fill ? (int64_t)nblocks : ceil_div((int64_t)P, ptile);
  hipLaunchKernelGGL(k_bucket_scatter, dim3((unsigned)tiles), dim3(CB), csr_bucket_scatter_lds(NB), st, rec, P,
                     rstart, K, cell_start, RB, DB, NB, bstart, (unsigned long long*)bcur, out, blk_fill, blk_pair,
                     blk_recs, blk_fill ? 2u : (uint32_t)rec_words, csr_bucket_stride());
}
void launch_csr_row_hist(const uint32_t* ent, const int64_t* tfirst, int64_t ntiles, int NB, const uint64_t* bstart,
                         int RB, int DB, int64_t N, uint32_t* rowcnt, hipStream_t st) {
  if (ntiles <= 0) return;
  hipLaunchKernelGGL(k_row_hist, dim3((unsigned)ntiles), dim3(CB), (size_t)(1 << RB) * 4, st, ent, tfirst, NB, bstart,
                     RB, DB, N, (int)csr_hist_tile(RB), rowcnt);
}
void launch_csr_row_scatter(const uint32_t* ent, const int64_t* tfirst, int64_t ntiles, int NB,
                            const uint64_t* bstart, int RB, int DB, int64_t N, const uint32_t* cpair,
                            const uint64_t* off, uint32_t* rowcur, uint32_t* heads, hipStream_t st) {
  if (ntiles <= 0) return;
  const int ept = csr_entries_per_thread(RB);
  auto k = ept == 8 ? k_row_scatter<8> : k_row_scatter<4>;
  hipLaunchKernelGGL(k, dim3((unsigned)ntiles), dim3(CB), csr_row_scatter_lds(RB), st, ent, tfirst, NB, bstart, RB, DB,
                     N, cpair, off, rowcur, heads);
}
void launch_csr_row_sort(const uint32_t* cpair, const int64_t* cell_start, const int32_t* ncells, const int2* cij,
                         const int32_t* ca, const uint32_t* rowcnt, const uint64_t* off, const uint32_t* heads,
                         int64_t N, int64_t max_pair_cells, int window_words, int num_cus, const int32_t* costK, uint32_t* col,
                         void* cost, uint64_t* rowq, hipStream_t st) {
  if (N <= 0) return;
  // the bitmap covers the largest pair's cells at once when they fit
  int win = (int)std::min<int64_t>(WIN_WORDS, std::max<int64_t>(1, (max_pair_cells + 31) / 32));
  if (window_words > 0) win = std::min(win, window_words);
  const size_t lds = (size_t)win * 4 + (size_t)SORT_WAVES * SORT_STAGE * 4;
  // persistent: two blocks per compute unit when their LDS fits (a bitmap
  // of up to 50 KiB, i.e. pairs of up to 400k cells), else one
  const int64_t grid = std::min<int64_t>(N, (int64_t)num_cus * (lds <= 76 * 1024 ? 2 : 1));
  if (costK)
    hipLaunchKernelGGL(k_row_sort<true>, dim3((unsigned)grid), dim3(SORT_B), lds, st, cpair, cell_start, ncells, cij, ca,
                       rowcnt, off, heads, N, win, costK, col, (int64_t*)cost,
                       (unsigned long long*)rowq);
  else
    hipLaunchKernelGGL(k_row_sort<false>, dim3((unsigned)grid), dim3(SORT_B), lds, st, cpair, cell_start, ncells, cij,
                       ca, rowcnt, off, heads, N, win, costK, col, (int32_t*)cost,
                       (unsigned long long*)rowq);
}
#define LAUNCH(kern, n, ...) \
  do { if ((n) > 0) hipLaunchKernelGGL(kern, dim3(blocks(n)), dim3(256), 0, st, __VA_ARGS__); } while (0)
void launch_csr_bflags(const int32_t* cb, int64_t N, uint32_t* flag, hipStream_t st) { LAUNCH(k_bflags, N, cb, N, flag); }
void launch_csr_row_deg(const uint32_t* cpair, const int64_t* cell_start, const int32_t* ncells, const int32_t* ca,
                        const int32_t* cb, const uint32_t* rowcnt, const uint32_t* bpos, int64_t N, uint64_t* deg,
                        hipStream_t st) {
  LAUNCH(k_row_deg, N, cpair, cell_start, ncells, ca, cb, rowcnt, bpos, N, deg);
}
void launch_csr_bdiag(const uint32_t* cpair, const int64_t* cell_start, const int32_t* ncells, const int2* cij,
                      const int32_t* ca, const int32_t* cb, const uint32_t* bpos, const uint64_t* off,
                      const PairArrays& P, int64_t N, const int32_t* costK, uint32_t* col, void* cost,
                      int64_t* supply, hipStream_t st) {
  if (costK) {
    LAUNCH(k_bdiag_rows<true>, N, cpair, cell_start, ncells, cij, ca, cb, bpos, off, P, N, costK, col, (int64_t*)cost,
           supply);
  } else {
    LAUNCH(k_bdiag_rows<false>, N, cpair, cell_start, ncells, cij, ca, cb, bpos, off, P, N, costK, col,
           (int32_t*)cost, supply);
  }
}

// Largest shifted cell coordinate of each diagram pair (the Euclidean cost
// scale): per-pair maxima over the cells.
__global__ void k_pair_xmax(const uint32_t* __restrict__ cpair, const int2* __restrict__ cij, int64_t N,
                            unsigned long long* __restrict__ xmax) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N) return;
  const int2 v = cij[g];
  const uint32_t p = cpair[g];
  const unsigned long long x = (unsigned long long)max(v.x, v.y);
  // one atomic per run of a pair inside the wave
  const uint32_t prev = __shfl_up(p, 1);
  unsigned long long m = x;
  for (int d = 1; d < WAVE; d <<= 1) {
    const unsigned long long o = __shfl_down(m, d);
    const uint32_t po = __shfl_down(p, d);
    if (lane_id() + d < WAVE && po == p && g + d < N && o > m) m = o;
  }
  if (lane_id() == 0 || prev != p) atomicMax(&xmax[p], m);
}
void launch_pair_xmax(const uint32_t* cpair, const int2* cij, int64_t N, uint64_t* xmax, hipStream_t st) {
  LAUNCH(k_pair_xmax, N, cpair, cij, N, (unsigned long long*)xmax);
}
void launch_csr_local_rowptr(const uint32_t* cpair, const int64_t* cell_start, const int32_t* ncells,
                             const uint64_t* off, int64_t N, int64_t* rp, hipStream_t st) {
  LAUNCH(k_local_rowptr, N, cpair, cell_start, ncells, off, N, rp);
}
void launch_csr_pair_arcs(const int64_t* cell_start, const uint64_t* off, int64_t K, int64_t nrows, uint64_t* out,
                          hipStream_t st) {
  LAUNCH(k_pair_arcs, K + 1, cell_start, off, K, nrows, out);
}

}  // namespace w1
