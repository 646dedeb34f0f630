// s-WSPD of the Morton radix tree (Alg. 4-6: for every internal node w,
// search the pair (w.left, w.right); output a pair when it is s-well-
// separated, otherwise split the node with the longer box side, ties
// splitting the second node).
//
// GPU organisation (differs from the paper's one-thread-per-internal-node
// scheme, whose work per thread ranges from one pair to millions):
//   1. expansion rounds: the root searches (w.left, w.right) of all internal
//      nodes form a work list; items whose subtrees are large are expanded
//      breadth-first, one level per round, until every item is either
//      separated or small (bounded subtree height sum and size product);
//      each round is compacted with scans so the item order is deterministic;
//   2. the final items are sorted by their first representative (Morton
//      order) and cut into chunks that never straddle two diagram pairs;
//   3. a persistent count pass and an identical emit pass: each wave takes a
//      chunk, its 64 lanes run depth-first searches with per-lane LDS
//      stacks, idle lanes refill from the chunk, and the pairs found in one
//      step are written contiguously at the wave's cursor (ballot + popcount).
//      The schedule inside a chunk depends only on the chunk, so both passes
//      see the same order and the output is deterministic.
//   Chunks are handed out from eight contiguous ranges, one per XCD
//   (workgroup b runs on XCD b mod 8), so each XCD's L2 holds a compact part
//   of the tree; an XCD that runs dry takes chunks from the other ranges.
#include "common.h"
#include "kernels.h"

namespace w1 {

namespace {

__device__ inline int4 node_box(const TreeView& T, int32_t r) {
  if (r >= 0) return T.ibox[r];
  const int2 c = T.cij[~r];
  return make_int4(c.x, c.y, c.x, c.y);
}
__device__ inline int32_t node_rep(const TreeView& T, int32_t r) { return r >= 0 ? T.iaux[r].z : ~r; }
__device__ inline int32_t node_height(const TreeView& T, int32_t r) { return r >= 0 ? T.iheight[r] : 0; }
__device__ inline int64_t node_size(const TreeView& T, int32_t r) {
  if (r < 0) return 1;
  const int4 a = T.iaux[r];
  return (int64_t)a.w - a.z + 1;
}
// Diagonal dominance of a node pair (optional pruning, not in the paper).
// Costs in units of g/2: an arc between cells p and q costs 2 max(|di|,|dj|)
// >= 2 dist(box U, box V), and a cell's arc to the diagonal costs j - i <=
// max j - min i of its box.  When 2 dist >= (U.maxj - U.mini) + (V.maxj -
// V.mini), every arc of the pair or of any pair below it in the recursion
// costs at least its two ends' diagonal arcs together, and leaving all of
// them out keeps the optimal flow cost: a flow path through such an arc can
// go from its source cell to the A-diagonal node and from the B-diagonal
// node to its sink cell instead (the distance to the diagonal is 1-Lipschitz
// along cell arcs), taking the flow off the zero-cost B->A diagonal arc.
// The test only gets truer further down (larger gaps, smaller boxes), so the
// recursion below a dominated pair is skipped.  Coordinates are below 2^30,
// so the sums fit in 32 unsigned bits.
__device__ inline bool dominated(int4 a, int4 b) {
  const int gi = max(a.x - b.z, b.x - a.z);
  const int gj = max(a.y - b.w, b.y - a.w);
  const uint32_t dist = (uint32_t)max(0, max(gi, gj));
  return 2u * dist >= (uint32_t)(a.w - a.x) + (uint32_t)(b.w - b.x);
}

// Metric of the separation test.  L-infinity: a node's diameter is its
// longest box side and (U, V) is separated when the box gap is at least s
// times the larger diameter.  Euclidean (the paper's balls): the diameter
// is the squared box diagonal and (U, V) is separated when the squared
// Euclidean box gap is at least s^2 times the larger one, in exact 128-bit
// integers.  The node with the larger diameter is split.
template <bool L2>
struct WMet;

template <>
struct WMet<false> {
  typedef int32_t D;
  __device__ static D diam(int4 b) { return max(b.z - b.x, b.w - b.y); }
  __device__ static bool sep(int4 a, D da, int4 b, D db, int s) {
    const int dist = max(max(max(a.x - b.z, b.x - a.z), max(a.y - b.w, b.y - a.w)), 0);
    return (int64_t)dist >= (int64_t)s * (int64_t)max(da, db);
  }
};

template <>
struct WMet<true> {
  typedef int64_t D;
  __device__ static D diam(int4 b) {
    const int64_t w = b.z - b.x, h = b.w - b.y;
    return w * w + h * h;
  }
  __device__ static bool sep(int4 a, D da, int4 b, D db, int s) {
    const int64_t gi = max(max(a.x - b.z, b.x - a.z), 0), gj = max(max(a.y - b.w, b.y - a.w), 0);
    const unsigned __int128 d2 = (unsigned __int128)(uint64_t)(gi * gi + gj * gj);
    return d2 >= (unsigned __int128)(uint64_t)((int64_t)s * s) * (uint64_t)(da > db ? da : db);
  }
};

template <bool L2>
__device__ inline bool separated_m(int4 a, int4 b, int s) {
  return WMet<L2>::sep(a, WMet<L2>::diam(a), b, WMet<L2>::diam(b), s);
}
// the first node is split (rather than the second) when its diameter is larger
template <bool L2>
__device__ inline bool split_first(int4 a, int4 b) {
  return WMet<L2>::diam(a) > WMet<L2>::diam(b);
}

__global__ void k_roots_flags(TreeView T, uint32_t* __restrict__ flag) {
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= T.N - 1) return;
  const int4 a = T.iaux[w];
  flag[w] = T.cpair[a.z] == T.cpair[a.w] ? 1u : 0u;
}

__global__ void k_roots_fill(TreeView T, const uint32_t* __restrict__ flag, const uint32_t* __restrict__ pos,
                             int2* __restrict__ items) {
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= T.N - 1 || !flag[w]) return;
  const int4 a = T.iaux[w];
  items[pos[w]] = make_int2(a.x, a.y);
}

// Item kinds of an expansion round: 0 dropped (diagonal-dominated, with
// pruning on), 1 kept (final: separated, or small enough for the traversal),
// 2 expanded (the node with the larger diameter is split in two).
__device__ inline uint32_t item_kind(const TreeView& T, int2 it, int4 bu, int4 bv, int s, int stack_depth,
                                     const int32_t* __restrict__ pair_cap, int prune, int l2) {
  if (prune && dominated(bu, bv)) return 0;
  const int64_t work_cap = pair_cap[T.cpair[node_rep(T, it.x)]];
  const bool small = node_height(T, it.x) + node_height(T, it.y) <= stack_depth - 1 &&
                     node_size(T, it.x) * node_size(T, it.y) <= work_cap;
  const bool keep = small || (l2 ? separated_m<true>(bu, bv, s) : separated_m<false>(bu, bv, s));
  return keep ? 1u : 2u;
}

// The two children of an expanded item, at next[q] and next[q + 1].
__device__ inline void expand_item(const TreeView& T, int2 it, int4 bu, int4 bv, int l2, int2* __restrict__ next,
                                   int64_t q) {
  if (l2 ? split_first<true>(bu, bv) : split_first<false>(bu, bv)) {
    const int4 a = T.iaux[it.x];
    next[q] = make_int2(a.x, it.y);
    next[q + 1] = make_int2(a.y, it.y);
  } else {
    const int4 a = T.iaux[it.y];
    next[q] = make_int2(it.x, a.x);
    next[q + 1] = make_int2(it.x, a.y);
  }
}

// One expansion round, counted: kept -> low word 1; expanded -> high word 2
// (its children); dropped -> 0.  The exclusive scan of these counts places
// every kept item and every child (k_scatter).
__global__ void k_classify(TreeView T, const int2* __restrict__ items, int64_t f, int s, int stack_depth,
                           const int32_t* __restrict__ pair_cap, int prune, int l2, uint64_t* __restrict__ cnt) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= f) return;
  const int2 it = items[x];
  const uint32_t kind = item_kind(T, it, node_box(T, it.x), node_box(T, it.y), s, stack_depth, pair_cap, prune, l2);
  cnt[x] = kind == 1 ? 1ull : kind == 2 ? (2ull << 32) : 0ull;
}

__global__ void k_scatter(TreeView T, const int2* __restrict__ items, int64_t f, const uint64_t* __restrict__ cnt,
                          const uint64_t* __restrict__ pos, int2* __restrict__ out_items, int64_t out_base,
                          int l2, int2* __restrict__ next) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= f) return;
  const int2 it = items[x];
  const uint64_t p = pos[x];
  if (cnt[x] == 0) return;  // dropped
  if (cnt[x] == 1ull) {
    out_items[out_base + (int64_t)(uint32_t)p] = it;
    return;
  }
  expand_item(T, it, node_box(T, it.x), node_box(T, it.y), l2, next, (int64_t)(p >> 32));
}

// Every expansion round of a small work list in one workgroup, so the host
// does not wait between rounds.  Tile by tile of XB items, in item order, the
// same exclusive scan of the same counts as k_classify / k_scatter places
// the kept items (appended to `kept`) and the children (the next frontier),
// so the work list is identical to the round-by-round one.  The frontiers
// alternate between fa and fb; the roots are only read, so the caller can
// run the rounds one by one from them when this kernel runs out of room.
// ctl[0]: items kept; ctl[1]: 0 done, 1 out of room, 2 more rounds than
// max_rounds.
constexpr int XB = 1024;
__global__ void __launch_bounds__(XB) k_expand_small(TreeView T, const int2* __restrict__ roots, int64_t f0, int s,
                                                     int stack_depth, const int32_t* __restrict__ pair_cap, int prune,
                                                     int l2, int max_rounds, int2* __restrict__ kept_out,
                                                     int64_t cap_kept, int2* fa, int2* fb, int64_t cap_front,
                                                     int64_t* __restrict__ ctl) {
  __shared__ uint64_t s_w[XB / WAVE];
  const int lane = lane_id(), wave = threadIdx.x / WAVE;
  const int2* src = roots;
  int2* dst = fa;
  int64_t f = f0, kept = 0;
  int status = 0;  // block-uniform
  for (int round = 0; f > 0 && status == 0; ++round) {
    if (round > max_rounds) {
      status = 2;
      break;
    }
    int64_t grown = 0;
    for (int64_t b0 = 0; b0 < f; b0 += XB) {
      const int64_t x = b0 + threadIdx.x;
      int2 it = make_int2(0, 0);
      int4 bu = make_int4(0, 0, 0, 0), bv = bu;
      uint32_t kind = 0;
      if (x < f) {
        it = src[x];
        bu = node_box(T, it.x);
        bv = node_box(T, it.y);
        kind = item_kind(T, it, bu, bv, s, stack_depth, pair_cap, prune, l2);
      }
      const uint64_t v = kind == 1 ? 1ull : kind == 2 ? (2ull << 32) : 0ull;
      uint64_t inc = v;
#pragma unroll
      for (int d = 1; d < WAVE; d <<= 1) {
        const uint64_t o = __shfl_up(inc, d);
        if (lane >= d) inc += o;
      }
      if (lane == WAVE - 1) s_w[wave] = inc;
      __syncthreads();
      uint64_t pre = 0, tot = 0;
      for (int w = 0; w < XB / WAVE; ++w) {
        const uint64_t t = s_w[w];
        if (w < wave) pre += t;
        tot += t;
      }
      __syncthreads();  // s_w is rewritten by the next tile
      const int64_t tk = (int64_t)(uint32_t)tot, tg = (int64_t)(tot >> 32);
      if (kept + tk > cap_kept || grown + tg > cap_front) {
        status = 1;
        break;
      }
      const uint64_t ex = pre + inc - v;
      if (kind == 1) kept_out[kept + (int64_t)(uint32_t)ex] = it;
      else if (kind == 2) expand_item(T, it, bu, bv, l2, dst, grown + (int64_t)(ex >> 32));
      kept += tk;
      grown += tg;
    }
    __syncthreads();  // the children written this round are read by other threads next round
    src = dst;
    dst = dst == fa ? fb : fa;
    f = grown;
  }
  if (threadIdx.x == 0) {
    ctl[0] = kept;
    ctl[1] = status;
  }
}

// Item keys.  (rep U, rep V) is canonical -- it depends only on the cells,
// not on node numbering -- and unique (the WSPD covers every cell pair once);
// the root search items are put in that order, the expansion rounds keep it,
// and the final work list is then stably sorted by rep U alone (Morton
// order, pair-major), so a pair's work list and hence its output order are
// the same alone or inside a batch.
__global__ void k_item_keys(TreeView T, const int2* __restrict__ items, int64_t m, int both,
                            uint64_t* __restrict__ keys) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= m) return;
  const uint64_t u = (uint32_t)node_rep(T, items[x].x);
  keys[x] = both ? ((u << 32) | (uint64_t)(uint32_t)node_rep(T, items[x].y)) : u;
}

__global__ void k_gather_items(const int2* __restrict__ src, const uint32_t* __restrict__ perm, int2* __restrict__ dst,
                               int64_t m) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x < m) dst[x] = src[perm[x]];
}

// Bounds of each diagram pair's run of work-list items, from the sorted
// keys (the first representative's cell, pair-major): first item writes
// lo[p], last writes hi[p].
__global__ void k_item_bounds(const uint32_t* __restrict__ cpair, const uint64_t* __restrict__ keys, int64_t m,
                              int64_t* __restrict__ lo, int64_t* __restrict__ hi) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= m) return;
  const uint32_t p = cpair[(uint32_t)keys[x]];
  if (x == 0 || cpair[(uint32_t)keys[x - 1]] != p) lo[p] = x;
  if (x == m - 1 || cpair[(uint32_t)keys[x + 1]] != p) hi[p] = x + 1;
}

// Chunk c of the work list: pair p is the last one with cstart[p] <= c (a
// pair's items are cut into ceil(items / chunk) chunks, in item order).
__global__ void k_chunks(const int32_t* __restrict__ cstart, int64_t K, const int64_t* __restrict__ item_start,
                         const int32_t* __restrict__ ipp, int64_t nch, int chunk, int32_t* __restrict__ chunk_first,
                         int32_t* __restrict__ chunk_end, int32_t* __restrict__ chunk_pair) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nch) return;
  int64_t a = 0, b = K;  // cstart[a] <= c < cstart[b]
  while (b - a > 1) {
    const int64_t h = (a + b) / 2;
    if (cstart[h] <= c) a = h;
    else b = h;
  }
  const int64_t x = item_start[a] + (c - cstart[a]) * (int64_t)chunk;
  const int64_t pend = item_start[a] + ipp[a];
  chunk_first[c] = (int32_t)x;
  chunk_end[c] = (int32_t)(x + chunk < pend ? x + chunk : pend);
  chunk_pair[c] = (int32_t)a;
}

// Traversal record, 32 bytes: int4 box (min i, min j, max i, max j) and
// int4 aux = (child base, local representative, rep i ^ 2^31, rep j ^ 2^31).
// Siblings are adjacent: record 0 is the root and the children of internal
// node g are records 2g + 1 (left) and 2g + 2 (right), so one offset locates
// both; the child base of a cell is -1 (cells are never split: a node pair
// of two cells is always separated).  The representative is the node's first
// cell, stored relative to its diagram pair's first cell; its coordinates
// carry a flipped sign bit so that unsigned order is signed order and the
// unsigned difference gives |a - b|.
struct Rec {
  int4 box, aux;
};

__device__ inline Rec rec_at(const int4* __restrict__ R, uint32_t i) {
  const int4* p = R + 2 * (size_t)i;
  return Rec{p[0], p[1]};
}
__device__ inline int64_t ref_index(const TreeView& T, int32_t r) { return r >= 0 ? r : (T.N - 1) + ~r; }

__device__ inline void put_rec(const TreeView& T, const int64_t* __restrict__ cell_start, int4* __restrict__ rec,
                               int32_t* __restrict__ rmap, int64_t at, int32_t r) {
  const int32_t rep = node_rep(T, r);
  const int2 c = T.cij[rep];
  rec[2 * at] = node_box(T, r);
  rec[2 * at + 1] = make_int4(r >= 0 ? r : -1, (int)(rep - cell_start[T.cpair[rep]]), (int)((uint32_t)c.x ^ 0x80000000u),
                              (int)((uint32_t)c.y ^ 0x80000000u));
  rmap[ref_index(T, r)] = (int32_t)at;
}

// One thread per internal node g writes the records of its two children
// (thread 0 also the root's) and the map from node reference to record.
__global__ void k_pack_nodes(TreeView T, const int64_t* __restrict__ cell_start, int4* __restrict__ rec,
                             int32_t* __restrict__ rmap) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= T.N - 1) return;
  const int4 a = T.iaux[g];
  put_rec(T, cell_start, rec, rmap, 2 * g + 1, a.x);
  put_rec(T, cell_start, rec, rmap, 2 * g + 2, a.y);
  if (g == 0) put_rec(T, cell_start, rec, rmap, 0, 0);
}

// Work entries of the passes (work list and stacks), int2:
//   x = record of the node to split next (P) | orient << 31,
//   y = record of the other node (O) | separated << 31,
// orient = 1 when P is the pair's first node U.  The split rule (longer box
// side, ties split the second node) is applied when an entry is made; a
// separated entry (fresh items only) is output as it is, U = P.
// Gathers the sorted work list (items[perm[x]]) and writes the entries.
__global__ void k_item_prep(TreeView T, const int2* __restrict__ items, const uint32_t* __restrict__ perm, int64_t m,
                            int s, const int32_t* __restrict__ rmap, int l2, int2* __restrict__ out) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= m) return;
  const int2 it = items[perm[x]];
  const int4 bu = node_box(T, it.x), bv = node_box(T, it.y);
  const int32_t ru = rmap[ref_index(T, it.x)], rv = rmap[ref_index(T, it.y)];
  int2 e;
  if (l2 ? separated_m<true>(bu, bv, s) : separated_m<false>(bu, bv, s))
    e = make_int2(ru | INT32_MIN, rv | INT32_MIN);
  else if (l2 ? split_first<true>(bu, bv) : split_first<false>(bu, bv))
    e = make_int2(ru | INT32_MIN, rv);
  else
    e = make_int2(rv, ru);
  out[x] = e;
}

// Packed split record of internal node g, 32 bytes: the boxes of its two
// children (left child's min i, min j, max i, max j, then the right child's)
// as eight 28-bit fields, coordinate k at bits [28k, 28k + 28) of words 0-6,
// and word 7 = the split index gamma (children are node gamma and gamma + 1).
// The count pass uses them when every cell coordinate of the launch is below
// 2^28: a split then reads 32 bytes (two loads) instead of both children's
// full records, and four split records share a 128-byte cache line.  The
// emit pass needs the children's representatives as well and reads their
// full records (one aligned 64-byte pair).
__global__ void k_pack_split(TreeView T, uint4* __restrict__ out) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= T.N - 1) return;
  const int4 a = T.iaux[g];
  const int4 b1 = node_box(T, a.x), b2 = node_box(T, a.y);
  const uint32_t v[8] = {(uint32_t)b1.x, (uint32_t)b1.y, (uint32_t)b1.z, (uint32_t)b1.w,
                         (uint32_t)b2.x, (uint32_t)b2.y, (uint32_t)b2.z, (uint32_t)b2.w};
  uint32_t d[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int o = 28 * k, w = o >> 5, sh = o & 31;
    d[w] |= v[k] << sh;
    if (sh > 4) d[w + 1] |= v[k] >> (32 - sh);
  }
  d[7] = (uint32_t)(a.x >= 0 ? a.x : ~a.x);
  out[2 * g] = make_uint4(d[0], d[1], d[2], d[3]);
  out[2 * g + 1] = make_uint4(d[4], d[5], d[6], d[7]);
}

__device__ inline void unpack_boxes(uint4 w0, uint4 w1, int4& b1, int4& b2) {
  const uint32_t M = 0x0fffffffu;
  b1.x = (int)(w0.x & M);
  b1.y = (int)(__builtin_amdgcn_alignbit(w0.y, w0.x, 28) & M);
  b1.z = (int)(__builtin_amdgcn_alignbit(w0.z, w0.y, 24) & M);
  b1.w = (int)(__builtin_amdgcn_alignbit(w0.w, w0.z, 20) & M);
  b2.x = (int)(__builtin_amdgcn_alignbit(w1.x, w0.w, 16) & M);
  b2.y = (int)(__builtin_amdgcn_alignbit(w1.y, w1.x, 12) & M);
  b2.z = (int)(__builtin_amdgcn_alignbit(w1.z, w1.y, 8) & M);
  b2.w = (int)(w1.z >> 4);
}

// Three-word pair record.  The vector type is 16 bytes in size (its store is
// 12), so records are addressed in 32-bit words, never by u32x3 arithmetic.
typedef uint32_t u32x3 __attribute__((ext_vector_type(3)));
typedef u32x3 u32x3_w __attribute__((aligned(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// Output pair (rep U, rep V, cost) of child / node aux c and the other node's
// aux o; orient = 1 when c is on the U side.  Cost = 2 * L-infinity distance
// of the representatives in grid units.
// (The Euclidean network's costs need more than 32 bits and are formed when
// the network's rows are sorted; its records carry 0 in the cost word.)
template <bool L2>
__device__ inline u32x3 make_emit(int4 c, int4 o, bool orient) {
  const uint32_t ci = (uint32_t)c.z, oi = (uint32_t)o.z, cj = (uint32_t)c.w, oj = (uint32_t)o.w;
  const uint32_t di = ci > oi ? ci - oi : oi - ci, dj = cj > oj ? cj - oj : oj - cj;
  return u32x3{(uint32_t)(orient ? c.y : o.y), (uint32_t)(orient ? o.y : c.y), L2 ? 0u : 2u * max(di, dj)};
}

// Checksum term of a pair record (u, v, cost) (see w1_result.pair_checksum).
__device__ inline uint64_t record_hash(u32x3 m) {
  const uint64_t x = ((uint64_t)m.x + 1) * 0x9E3779B97F4A7C15ull + ((uint64_t)m.y + 1);
  return (x * 0xC2B2AE3D27D4EB4Full + (uint64_t)m.z) * 0x165667B19E3779F9ull;
}

// Lanes below this one whose bit is set in m, plus add.
__device__ inline uint32_t lanes_set_below(uint64_t m, uint32_t add) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, add));
}

// Count pass (EMIT = false) and emit pass (EMIT = true) of the WSPD search
// over the chunks of the work list.  Lane state: a node pair known to be not
// separated, held as (P, O, orient): the aux of P, the node to split (its
// child base, and its representative, which is also its left child's), and
// O's record.  A split of P reads both children's records (one aligned
// 64-byte pair, four loads); COMPACT reads P's packed 32-byte split record
// instead (two loads).  Both hold the same boxes and child bases, so the
// pairs are the same.  The representatives a COMPACT emit pass needs follow
// from the split index gamma: the left child starts where P starts (P's
// representative), the right child at cell gamma + 1.  Its records are
// (u, v) without the cost (the network's costs come from the cells when its
// rows are sorted), 8 bytes each.  A step first lets every lane without a pair acquire an
// entry (pop its LDS stack, else take a fresh item from the chunk); a
// separated fresh item is output at once.  Then each lane with a pair loads
// both children of P (adjacent records), tests both child pairs against O
// (one dependent memory round trip resolves two recursion nodes): separated
// child pairs are output, the first non-separated one becomes the lane's pair
// and a second one goes on the stack.  At most two pairs per lane per step,
// written as 12-byte records at the wave cursor in (slot, lane) order, so the
// order depends only on the chunk.  Loop control lives in wave-uniform
// scalars.
template <bool EMIT, bool COMPACT, bool PRUNE, bool L2, bool BLOCKS>
__global__ void __launch_bounds__(256) k_wspd(const int4* __restrict__ R, const uint4* __restrict__ SR,
                                              const int2* __restrict__ items,
                                              const int32_t* __restrict__ chunk_first, const int32_t* __restrict__ chunk_end,
                                              const int32_t* __restrict__ xcd_range, uint32_t* __restrict__ xcd_ctr, int s,
                                              int stack_depth, int64_t step_cap, uint64_t* __restrict__ chunk_cnt,
                                              const uint64_t* __restrict__ chunk_off, uint32_t* __restrict__ out,
                                              int32_t* __restrict__ err, BucketHist bh, StreamOut so, BlockOut bo,
                                              int chunk_stride) {
  static_assert(!(COMPACT && BLOCKS), "blocked output reads the full records");
  static_assert(EMIT || !BLOCKS, "blocked output is an emit-pass mode");
  extern __shared__ int2 s_stack[];
  const int wave = threadIdx.x / WAVE, lane = lane_id();
  int2* stk = s_stack + (size_t)wave * stack_depth * WAVE + lane;  // entry e at stk[e * WAVE]
  // emit pass: arcs per tail bucket of the network's row partition (both
  // orientations of every pair), counted in LDS and added up at the end
  uint32_t* s_hist = (uint32_t*)(s_stack + (size_t)4 * stack_depth * WAVE);
  if (EMIT) {
    for (int b = threadIdx.x; b < bh.NB; b += blockDim.x) s_hist[b] = 0;
    __syncthreads();
  }
  // blocked output (network path): the wave's current block, wave-uniform
  int blk = -1, bpair = -1;
  uint32_t bleft = 0;
  uint32_t* bptr = nullptr;  // where the block's next record goes (kept across chunks)
  bool dead = false;
  auto retire = [&]() {
    if (blk >= 0 && lane == 0) {
      const uint32_t f = bo.block - bleft;
      bo.fill[blk] = f;
      bo.pair[blk] = (uint32_t)bpair;
      atomicAdd(&bo.pair_count[bpair], (unsigned long long)f);
    }
    blk = -1;
    bleft = 0;
  };
  const uint64_t sbase = so.base_dev ? (uint64_t)*so.base_dev : (uint64_t)so.base;
  const int xcd = blockIdx.x & 7;
  for (int probe = 0; probe < 8; ++probe) {
    const int xr = (xcd + probe) & 7;
    const int r0 = xcd_range[xr], r1 = xcd_range[xr + 1];
    for (;;) {
      // every lane takes part in the fetch (lane 0 adds 1, the others 0), so
      // there is no lane-divergent region in the chunk loop
      const uint32_t t = atomicAdd(&xcd_ctr[xr], lane == 0 ? 1u : 0u);
      const int k = (int)__builtin_amdgcn_readfirstlane(t) * chunk_stride + r0;
      if (k >= r1) break;
      int next = __builtin_amdgcn_readfirstlane(chunk_first[k]);
      const int end = __builtin_amdgcn_readfirstlane(chunk_end[k]);
      const int kp = BLOCKS ? bo.chunk_pair[k] : 0;
      if (BLOCKS && blk >= 0 && kp != bpair) retire();  // a block holds one diagram pair
      // records go at the chunk's counted offset, or on in the wave's block
      uint32_t* obase = !EMIT    ? nullptr
                        : BLOCKS  ? bptr
                        : so.slot ? out + (COMPACT ? 2 : 3) * ((uint64_t)k * (uint64_t)so.slot)
                        : COMPACT ? out + 2 * (chunk_off[k] - sbase)
                                  : out + 3 * (chunk_off[k] - sbase);
      uint64_t h1 = 0, h2 = 0;  // streamed emission: the lane's checksum terms
      const uint64_t cs = EMIT && (COMPACT || bh.NB > 0) ? (uint64_t)bh.cell_start[bh.chunk_pair[k]] : 0;
      uint64_t cursor = 0;
      typedef typename WMet<L2>::D Diam;
      bool has = false, overflow = false, runaway = false, orient = false;
      int sp = 0, oid = 0;
      Diam od = 0;
      int4 ob = make_int4(0, 0, 0, 0), oa = ob, pa = ob;
      for (int64_t step = 0;; ++step) {
        if (step > step_cap) {  // beyond any chunk's possible work: give up, report
          runaway = true;
          break;
        }
        // acquire: stack first, then fresh items in lane order
        const bool want = !has;
        const uint64_t need = __ballot(want && sp == 0);
        const int avail = end - next;
        bool got = false;
        int2 q = make_int2(0, 0);
        if (want) {
          if (sp > 0) {
            --sp;
            q = stk[sp * WAVE];
            got = true;
          } else {
            const int r = (int)lanes_set_below(need, 0u);
            if (r < avail) {
              q = items[next + r];
              got = true;
            }
          }
        }
        const int took = __popcll(need);
        next += took < avail ? took : (avail > 0 ? avail : 0);
        if (got) {
          oid = q.y & 0x7fffffff;
          const Rec O = rec_at(R, (uint32_t)oid);
          pa = R[2 * (size_t)(uint32_t)(q.x & 0x7fffffff) + 1];
          ob = O.box;
          oa = O.aux;
          orient = q.x < 0;
        }
        if (__ballot(has || got) == 0) break;
        bool e1 = false, e2 = false;
        u32x3 m1, m2;
        if (got) {
          if (q.y < 0) {
            e1 = true;
            if (EMIT) m1 = make_emit<L2>(pa, oa, orient);
          } else {
            has = true;
            od = WMet<L2>::diam(ob);
          }
        }
        if (has) {
          const uint32_t c1 = 2 * (uint32_t)pa.x + 1;
          Rec C1, C2;
          if (COMPACT) {
            const uint4* ps = SR + 2 * (size_t)(uint32_t)pa.x;
            const uint4 w0 = ps[0], w1 = ps[1];
            unpack_boxes(w0, w1, C1.box, C2.box);
            const int gamma = (int)w1.w;
            C1.aux = make_int4(gamma, EMIT ? pa.y : 0, 0, 0);
            C2.aux = make_int4(gamma + 1, EMIT ? (int)((int64_t)gamma + 1 - (int64_t)cs) : 0, 0, 0);
          } else {
            const int4* pc = R + 2 * (size_t)c1;  // both children: 64 contiguous, aligned bytes
            C1 = Rec{pc[0], pc[1]};
            C2 = Rec{pc[2], pc[3]};
          }
          const Diam d1 = WMet<L2>::diam(C1.box), d2 = WMet<L2>::diam(C2.box);
          const bool s1 = WMet<L2>::sep(C1.box, d1, ob, od, s), s2 = WMet<L2>::sep(C2.box, d2, ob, od, s);
          if (EMIT) {
            m1 = make_emit<L2>(C1.aux, oa, orient);
            m2 = make_emit<L2>(C2.aux, oa, orient);
          }
          // a child pair is done when separated (output unless dominated) or
          // dominated (pruning: no output, nothing below it)
          const bool x1 = PRUNE && dominated(C1.box, ob), x2 = PRUNE && dominated(C2.box, ob);
          e1 = s1 && !x1;
          e2 = s2 && !x2;
          const bool r1 = s1 || x1, r2 = s2 || x2;
          if (!r1 && !r2) {  // (C2, O) goes on the stack, split rule applied
            const bool split2 = orient ? d2 > od : d2 >= od;
            const int c2 = (int)(c1 + 1);
            const int2 e = split2 ? make_int2(c2 | (orient ? INT32_MIN : 0), oid)
                                  : make_int2(oid | (orient ? 0 : INT32_MIN), c2);
            if (sp < stack_depth) {
              stk[sp * WAVE] = e;
              ++sp;
            } else {
              overflow = true;
            }
          }
          if (!r1 || !r2) {  // the lane's next pair: (first child not done, O)
            const bool first = !r1;
            const Diam dn = first ? d1 : d2;
            const int4 na = first ? C1.aux : C2.aux;
            if (orient ? dn > od : dn >= od) {
              pa = na;
            } else {  // O is split next; the child takes O's place
              pa = oa;
              ob = first ? C1.box : C2.box;
              oa = na;
              oid = (int)(first ? c1 : c1 + 1);
              od = dn;
              orient = !orient;
            }
          } else {
            has = false;
          }
        }
        const uint64_t b1 = __ballot(e1), b2 = __ballot(e2);
        const uint32_t n1 = (uint32_t)__popcll(b1), n2 = (uint32_t)__popcll(b2);
        if (EMIT) {
          // streaming (non-temporal) 12-byte stores: the output is written
          // once and must not evict the tree from L2
          bool wr = true;
          if (BLOCKS) {  // blocked output: a fresh block when this step's records do not fit
            const uint32_t n = n1 + n2;
            if (n > bleft && !dead) {
              retire();
              uint32_t b = 0;
              if (lane == 0) b = atomicAdd(bo.nblocks, 1u);
              b = (uint32_t)__shfl((int)b, 0);
              if (b < bo.max_blocks) {
                blk = (int)b;
                bpair = kp;
                bleft = bo.block;
                obase = bo.base + 2 * (size_t)b * bo.block;
              } else {
                dead = true;
                if (lane == 0) atomicOr(bo.overflow, 1);
              }
            }
            wr = !dead;
            if (wr) bleft -= n;
          }
          if (!BLOCKS && so.slot && cursor + n1 + n2 > (uint64_t)so.slot) {  // beyond the chunk's slot
            wr = false;
            overflow = true;
          }
          if (wr && (BLOCKS || COMPACT)) {  // (u, v): the network's costs come from the cells
            if (e1) __builtin_nontemporal_store(u32x2{m1.x, m1.y}, (u32x2*)(obase + 2 * lanes_set_below(b1, 0u)));
            if (e2) __builtin_nontemporal_store(u32x2{m2.x, m2.y}, (u32x2*)(obase + 2 * lanes_set_below(b2, n1)));
            obase += 2 * (n1 + n2);
          } else if (wr && !BLOCKS && !COMPACT) {
            if (e1) __builtin_nontemporal_store(m1, (u32x3_w*)(obase + 3 * lanes_set_below(b1, 0u)));
            if (e2) __builtin_nontemporal_store(m2, (u32x3_w*)(obase + 3 * lanes_set_below(b2, n1)));
            obase += 3 * (n1 + n2);
          }
          if (!COMPACT && so.chunk_sum) {
            if (e1) {
              const uint64_t h = record_hash(m1);
              h1 += h;
              h2 += h * h;
            }
            if (e2) {
              const uint64_t h = record_hash(m2);
              h1 += h;
              h2 += h * h;
            }
          }
          if (bh.NB > 0) {
            if (e1) {
              atomicAdd(&s_hist[(uint32_t)((cs + m1.x) >> bh.RB)], 1u);
              atomicAdd(&s_hist[(uint32_t)((cs + m1.y) >> bh.RB)], 1u);
            }
            if (e2) {
              atomicAdd(&s_hist[(uint32_t)((cs + m2.x) >> bh.RB)], 1u);
              atomicAdd(&s_hist[(uint32_t)((cs + m2.y) >> bh.RB)], 1u);
            }
          }
        }
        cursor += n1 + n2;
      }
      if (BLOCKS) bptr = obase;
      const bool bad = runaway || __ballot(overflow) != 0;
      if (bad) atomicOr(err, 1);
      if (!EMIT || so.slot) chunk_cnt[k] = cursor;  // same value from every lane
      if (EMIT && so.chunk_sum) {
        for (int d = WAVE / 2; d > 0; d >>= 1) {
          h1 += __shfl_xor(h1, d);
          h2 += __shfl_xor(h2, d);
        }
        if (lane == 0) {
          so.chunk_sum[2 * k] = h1;
          so.chunk_sum[2 * k + 1] = h2;
        }
      }
    }
  }
  if (BLOCKS) retire();
  if (EMIT && bh.NB > 0) {
    __syncthreads();
    for (int b = threadIdx.x; b < bh.NB; b += blockDim.x)
      if (s_hist[b]) atomicAdd((unsigned long long*)&bh.count[b], (unsigned long long)s_hist[b]);
  }
}

// Per diagram pair: first output position (the first chunk's offset) and
// pair count (end of its last chunk minus that).  Chunks are pair-major.
__global__ void k_pair_bounds(const uint64_t* __restrict__ chunk_cnt, const uint64_t* __restrict__ chunk_off,
                              const int32_t* __restrict__ chunk_pair, int64_t nchunks, uint64_t* __restrict__ pair_start,
                              uint64_t* __restrict__ pair_end) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nchunks) return;
  const int32_t p = chunk_pair[c];
  if (c == 0 || chunk_pair[c - 1] != p) pair_start[p] = chunk_off[c];
  if (c == nchunks - 1 || chunk_pair[c + 1] != p) pair_end[p] = chunk_off[c] + chunk_cnt[c];
}

__global__ void k_pair_counts(const uint64_t* __restrict__ pair_start, const uint64_t* __restrict__ pair_end, int64_t K,
                              uint64_t* __restrict__ npairs) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < K) npairs[p] = pair_end[p] > pair_start[p] ? pair_end[p] - pair_start[p] : 0;
}

__global__ void k_compact_slots(const uint32_t* __restrict__ src, const uint64_t* __restrict__ cnt,
                                const uint64_t* __restrict__ off, int64_t slot, int w, uint32_t* __restrict__ dst) {
  const int64_t k = blockIdx.x;
  // a chunk never outgrows its slot (the emit pass reports one that would,
  // and the call fails); the clamp keeps the reads inside the slot anyway
  const int64_t n = (int64_t)min(cnt[k], (uint64_t)slot) * w;
  const uint32_t* s = src + (uint64_t)k * (uint64_t)slot * (uint64_t)w;
  uint32_t* d = dst + off[k] * (uint64_t)w;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) d[i] = s[i];
}

__global__ void k_stream_next(const int32_t* __restrict__ run_xr, const int64_t* __restrict__ run_base, int nruns,
                              int32_t* __restrict__ ctr, int32_t* __restrict__ xr, int64_t* __restrict__ base,
                              uint32_t* __restrict__ xc) {
  const int r = *ctr;  // every thread reads it before thread 0 advances it
  __syncthreads();
  const int t = threadIdx.x;
  if (t < 9) xr[t] = r < nruns ? run_xr[9 * r + t] : 0;
  if (t < 8) xc[t] = 0;
  if (t == 0) {
    *base = r < nruns ? run_base[r] : 0;
    *ctr = r + 1;
  }
}

inline unsigned blocks(int64_t n, int bs = 256) { return (unsigned)(n > 0 ? ceil_div(n, bs) : 1); }

}  // namespace

#define LAUNCH(kern, n, ...) \
  do { if ((n) > 0) hipLaunchKernelGGL(kern, dim3(blocks(n)), dim3(256), 0, st, __VA_ARGS__); } while (0)

void launch_pack_nodes(const TreeView& T, const int64_t* cell_start, int4* rec, int32_t* rmap, hipStream_t st) {
  LAUNCH(k_pack_nodes, T.N - 1, T, cell_start, rec, rmap);
}
void launch_pack_split(const TreeView& T, uint4* out, hipStream_t st) { LAUNCH(k_pack_split, T.N - 1, T, out); }
void launch_item_prep(const TreeView& T, const int2* items, const uint32_t* perm, int64_t m, int s, const int32_t* rmap,
                      bool l2, int2* out, hipStream_t st) {
  LAUNCH(k_item_prep, m, T, items, perm, m, s, rmap, l2 ? 1 : 0, out);
}
void launch_wspd_roots_flags(const TreeView& T, uint32_t* flag, hipStream_t st) { LAUNCH(k_roots_flags, T.N - 1, T, flag); }
void launch_wspd_roots_fill(const TreeView& T, const uint32_t* flag, const uint32_t* pos, int2* items, hipStream_t st) {
  LAUNCH(k_roots_fill, T.N - 1, T, flag, pos, items);
}
void launch_wspd_classify(const TreeView& T, const int2* items, int64_t f, int s, const WspdTuning& tun,
                          const int32_t* pair_cap, bool prune, bool l2, uint64_t* cnt, hipStream_t st) {
  LAUNCH(k_classify, f, T, items, f, s, tun.stack_depth, pair_cap, prune ? 1 : 0, l2 ? 1 : 0, cnt);
}
void launch_wspd_scatter(const TreeView& T, const int2* items, int64_t f, const uint64_t* cnt, const uint64_t* pos,
                         int2* out_items, int64_t out_base, bool l2, int2* next, hipStream_t st) {
  LAUNCH(k_scatter, f, T, items, f, cnt, pos, out_items, out_base, l2 ? 1 : 0, next);
}
void launch_wspd_expand_small(const TreeView& T, const int2* roots, int64_t f0, int s, const WspdTuning& tun,
                              const int32_t* pair_cap, bool prune, bool l2, int max_rounds, int2* kept,
                              int64_t cap_kept, int2* fa, int2* fb, int64_t cap_front, int64_t* ctl, hipStream_t st) {
  hipLaunchKernelGGL(k_expand_small, dim3(1), dim3(XB), 0, st, T, roots, f0, s, tun.stack_depth, pair_cap,
                     prune ? 1 : 0, l2 ? 1 : 0, max_rounds, kept, cap_kept, fa, fb, cap_front, ctl);
}
void launch_item_keys(const TreeView& T, const int2* items, int64_t m, bool both, uint64_t* keys, hipStream_t st) {
  LAUNCH(k_item_keys, m, T, items, m, both ? 1 : 0, keys);
}
void launch_gather_items(const int2* src, const uint32_t* perm, int2* dst, int64_t m, hipStream_t st) {
  LAUNCH(k_gather_items, m, src, perm, dst, m);
}
void launch_item_bounds(const uint32_t* cpair, const uint64_t* keys, int64_t m, int64_t* lo, int64_t* hi,
                        hipStream_t st) {
  LAUNCH(k_item_bounds, m, cpair, keys, m, lo, hi);
}
void launch_chunks(const int32_t* cstart, int64_t K, const int64_t* item_start, const int32_t* ipp, int64_t nch,
                   int chunk, int32_t* chunk_first, int32_t* chunk_end, int32_t* chunk_pair, hipStream_t st) {
  LAUNCH(k_chunks, nch, cstart, K, item_start, ipp, nch, chunk, chunk_first, chunk_end, chunk_pair);
}
int launch_wspd_pass(bool emit, const TreeView& T, const uint4* split_recs, const int2* items,
                      const int32_t* chunk_first, const int32_t* chunk_end, int64_t nchunks, const int32_t* xcd_range,
                      uint32_t* xcd_ctr, int s, const WspdTuning& tun, uint64_t* chunk_cnt, const uint64_t* chunk_off,
                      uint32_t* out, int32_t* err, bool prune, bool l2, const BucketHist& bh, const StreamOut& so,
                      const BlockOut& bo, int chunk_stride, int num_cus, hipStream_t st) {
  if (nchunks <= 0) return 0;
  // persistent blocks of 4 waves, but no more than the chunks need: every
  // wave starts by probing the 8 shared chunk counters, and thousands of
  // idle waves doing so cost a short work list ~0.4 ms per pass
  int64_t grid = (int64_t)num_cus * tun.blocks_per_cu;
  const int64_t cstride = chunk_stride > 0 ? chunk_stride : 1;
  grid = std::min(grid, ceil_div(ceil_div(nchunks, cstride), (int64_t)4));
  grid = std::max<int64_t>(8, ((grid + 7) / 8) * 8);
  const size_t lds = (size_t)4 * tun.stack_depth * WAVE * sizeof(int2) + (emit ? (size_t)bh.NB * 4 : 0);
  // A chunk's items each have at most work_cap leaf pairs, hence fewer than
  // 2 work_cap recursion nodes; every wave step resolves at least one.
  const int64_t step_cap = (int64_t)tun.chunk_items * (2 * (int64_t)tun.work_cap + 2) + 1024;
  // the emit pass reads the packed split records only when it writes
  // (u, v) records for the network (it needs the chunks' first cells, which
  // come with the bucket histogram); with checksums or blocks it reads the
  // children's full records
  const bool blocks = emit && bo.base;
  const bool packed = split_recs && (!emit || (!blocks && !so.chunk_sum && bh.NB > 0));
  auto k = l2 ? (blocks ? k_wspd<true, false, false, true, true>
                 : emit ? (packed ? k_wspd<true, true, false, true, false> : k_wspd<true, false, false, true, false>)
                        : (packed ? k_wspd<false, true, false, true, false> : k_wspd<false, false, false, true, false>))
         : prune ? (blocks ? k_wspd<true, false, true, false, true>
                    : emit ? (packed ? k_wspd<true, true, true, false, false> : k_wspd<true, false, true, false, false>)
                           : (packed ? k_wspd<false, true, true, false, false>
                                     : k_wspd<false, false, true, false, false>))
                 : (blocks ? k_wspd<true, false, false, false, true>
                    : emit ? (packed ? k_wspd<true, true, false, false, false> : k_wspd<true, false, false, false, false>)
                           : (packed ? k_wspd<false, true, false, false, false>
                                     : k_wspd<false, false, false, false, false>));
  hipLaunchKernelGGL(k, dim3((unsigned)grid), dim3(256), lds, st, T.inode, split_recs, items, chunk_first, chunk_end,
                     xcd_range, xcd_ctr, s, tun.stack_depth, step_cap, chunk_cnt, chunk_off, out, err,
                     emit ? bh : BucketHist{}, emit ? so : StreamOut{}, emit ? bo : BlockOut{},
                     chunk_stride > 0 ? chunk_stride : 1);
  return !emit ? 0 : (blocks || packed) ? 2 : 3;
}
void launch_compact_slots(const uint32_t* src, const uint64_t* cnt, const uint64_t* off, int64_t nch, int64_t slot,
                          int w, uint32_t* dst, hipStream_t st) {
  if (nch > 0) hipLaunchKernelGGL(k_compact_slots, dim3((unsigned)nch), dim3(256), 0, st, src, cnt, off, slot, w, dst);
}
void launch_stream_next(const int32_t* run_xr, const int64_t* run_base, int nruns, int32_t* ctr, int32_t* xr,
                        int64_t* base, uint32_t* xc, hipStream_t st) {
  hipLaunchKernelGGL(k_stream_next, dim3(1), dim3(64), 0, st, run_xr, run_base, nruns, ctr, xr, base, xc);
}
void launch_pair_totals(const uint64_t* chunk_cnt, const uint64_t* chunk_off, const int32_t* chunk_pair,
                        int64_t nchunks, uint64_t* pair_start, uint64_t* pair_end, uint64_t* npairs, int64_t K,
                        hipStream_t st) {
  LAUNCH(k_pair_bounds, nchunks, chunk_cnt, chunk_off, chunk_pair, nchunks, pair_start, pair_end);
  LAUNCH(k_pair_counts, K, pair_start, pair_end, K, npairs);
}

}  // namespace w1
