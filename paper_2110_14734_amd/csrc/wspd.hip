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
__device__ inline int32_t box_diam(int4 b) { return max(b.z - b.x, b.w - b.y); }
__device__ inline bool separated(int4 a, int4 b, int s) {
  const int gi = max(a.x - b.z, b.x - a.z);
  const int gj = max(a.y - b.w, b.y - a.w);
  const int dist = max(0, max(gi, gj));
  return (int64_t)dist >= (int64_t)s * (int64_t)max(box_diam(a), box_diam(b));
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

// Item kinds of an expansion round: kept (final or separated) -> low word
// count 1; expanded -> high word count 2.
__global__ void k_classify(TreeView T, const int2* __restrict__ items, int64_t f, int s, int stack_depth,
                           int64_t work_cap, uint64_t* __restrict__ cnt) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= f) return;
  const int2 it = items[x];
  const bool small = node_height(T, it.x) + node_height(T, it.y) <= stack_depth - 1 &&
                     node_size(T, it.x) * node_size(T, it.y) <= work_cap;
  const bool keep = small || separated(node_box(T, it.x), node_box(T, it.y), s);
  cnt[x] = keep ? 1ull : (2ull << 32);
}

__global__ void k_scatter(TreeView T, const int2* __restrict__ items, int64_t f, const uint64_t* __restrict__ cnt,
                          const uint64_t* __restrict__ pos, int2* __restrict__ out_items, int64_t out_base,
                          int2* __restrict__ next) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= f) return;
  const int2 it = items[x];
  const uint64_t p = pos[x];
  if (cnt[x] == 1ull) {
    out_items[out_base + (int64_t)(uint32_t)p] = it;
    return;
  }
  const int64_t q = (int64_t)(p >> 32);
  const int4 bu = node_box(T, it.x), bv = node_box(T, it.y);
  if (box_diam(bu) > box_diam(bv)) {
    const int4 a = T.iaux[it.x];
    next[q] = make_int2(a.x, it.y);
    next[q + 1] = make_int2(a.y, it.y);
  } else {
    const int4 a = T.iaux[it.y];
    next[q] = make_int2(it.x, a.x);
    next[q + 1] = make_int2(it.x, a.y);
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

// Bounds of each diagram pair's run of work-list items (items are sorted
// pair-major): first item writes lo[p], last writes hi[p].
__global__ void k_item_bounds(TreeView T, const int2* __restrict__ items, int64_t m, int64_t* __restrict__ lo,
                              int64_t* __restrict__ hi) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= m) return;
  const uint32_t p = T.cpair[node_rep(T, items[x].x)];
  if (x == 0 || T.cpair[node_rep(T, items[x - 1].x)] != p) lo[p] = x;
  if (x == m - 1 || T.cpair[node_rep(T, items[x + 1].x)] != p) hi[p] = x + 1;
}

__global__ void k_chunk_heads(TreeView T, const int2* __restrict__ items, int64_t m, const int64_t* __restrict__ item_start,
                              int chunk, uint32_t* __restrict__ head) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= m) return;
  const uint32_t p = T.cpair[node_rep(T, items[x].x)];
  head[x] = ((x - item_start[p]) % chunk) == 0 ? 1u : 0u;
}

__global__ void k_chunk_fill(TreeView T, const int2* __restrict__ items, int64_t m, const int64_t* __restrict__ item_start,
                             const int32_t* __restrict__ ipp, const uint32_t* __restrict__ head,
                             const uint32_t* __restrict__ cid, int chunk, int32_t* __restrict__ chunk_first,
                             int32_t* __restrict__ chunk_end, int32_t* __restrict__ chunk_pair) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= m || !head[x]) return;
  const uint32_t p = T.cpair[node_rep(T, items[x].x)];
  const uint32_t c = cid[x];
  const int64_t pend = item_start[p] + ipp[p];
  chunk_first[c] = (int32_t)x;
  chunk_end[c] = (int32_t)(x + chunk < pend ? x + chunk : pend);
  chunk_pair[c] = (int32_t)p;
}

// Packed node record for the traversal, 32 bytes, one format for internal
// nodes and cells: int4 box (min i, min j, max i, max j) and int4 aux =
// (representative cell, split | left-is-cell << 30 | right-is-cell << 31,
// representative i, representative j).  Internal node r has split g: its
// children are g and g + 1 (cells or internal nodes, per the two flags).
// Record index: internal node r -> r, cell c -> (N - 1) + c.
struct Rec {
  int4 box, aux;
};

__device__ inline Rec load_rec(const int4* __restrict__ R, int32_t r, int32_t nint) {
  const int64_t i = r >= 0 ? (int64_t)r : (int64_t)nint + ~r;
  const int4* p = R + 2 * i;
  return Rec{p[0], p[1]};
}
__device__ inline int32_t rec_left(const Rec& q) {
  const uint32_t f = (uint32_t)q.aux.y;
  const int32_t g = (int32_t)(f & 0x3fffffffu);
  return (f >> 30) & 1u ? ~g : g;
}
__device__ inline int32_t rec_right(const Rec& q) {
  const uint32_t f = (uint32_t)q.aux.y;
  const int32_t g = (int32_t)(f & 0x3fffffffu) + 1;
  return (f >> 31) ? ~g : g;
}

__global__ void k_pack_nodes(TreeView T, int4* __restrict__ rec) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nint = T.N - 1;
  if (r >= nint + T.N) return;
  if (r < nint) {
    const int4 a = T.iaux[r];  // left, right, lo, hi
    const int32_t g = a.x >= 0 ? a.x : ~a.x;
    const uint32_t f = (uint32_t)g | (a.x < 0 ? 1u << 30 : 0u) | (a.y < 0 ? 1u << 31 : 0u);
    const int2 c = T.cij[a.z];
    rec[2 * r] = T.ibox[r];
    rec[2 * r + 1] = make_int4(a.z, (int)f, c.x, c.y);
  } else {
    const int32_t cell = (int32_t)(r - nint);
    const int2 c = T.cij[cell];
    rec[2 * r] = make_int4(c.x, c.y, c.x, c.y);
    rec[2 * r + 1] = make_int4(cell, 0, c.x, c.y);
  }
}

// Three-word pair record.  The vector type is 16 bytes in size (its store is
// 12), so records are addressed in 32-bit words, never by u32x3 arithmetic.
typedef uint32_t u32x3 __attribute__((ext_vector_type(3)));
typedef u32x3 u32x3_w __attribute__((aligned(4)));

// One emitted pair: (rep U - cell base, rep V - cell base, cost).
__device__ inline u32x3 make_emit(const Rec& a, const Rec& b, int64_t cs) {
  const int c = 2 * max(abs(a.aux.z - b.aux.z), abs(a.aux.w - b.aux.w));
  return u32x3{(uint32_t)(a.aux.x - cs), (uint32_t)(b.aux.x - cs), (uint32_t)c};
}

// Count pass (EMIT = false) and emit pass (EMIT = true) of the WSPD search
// over the chunks of the work list.  Lane state: a node pair known to be not
// separated ("current"), or none.  A step first lets every lane without a
// current pair acquire one (pop its LDS stack, else take a fresh item from
// the chunk) through a single record-load path; fresh items are tested.  Then
// each current pair splits the node with the longer box side, loads both
// children and tests both child pairs (one dependent memory round trip
// resolves two recursion nodes): separated child pairs are emitted, a
// non-separated one becomes current and a second one goes on the stack.  At
// most two pairs per lane per step, written as 12-byte records at the wave
// cursor in (slot, lane) order, so the order depends only on the chunk.
// Loop control lives in wave-uniform scalars.
template <bool EMIT>
__global__ void __launch_bounds__(256) k_wspd(TreeView T, const int2* __restrict__ items,
                                              const int32_t* __restrict__ chunk_first, const int32_t* __restrict__ chunk_end,
                                              const int32_t* __restrict__ chunk_pair, const int32_t* __restrict__ xcd_range,
                                              uint32_t* __restrict__ xcd_ctr, int s, int stack_depth, int64_t step_cap,
                                              uint64_t* __restrict__ chunk_cnt, const uint64_t* __restrict__ chunk_off,
                                              const int64_t* __restrict__ cell_start, uint32_t* __restrict__ out,
                                              int32_t* __restrict__ err) {
  extern __shared__ int2 s_stack[];
  const int wave = threadIdx.x / WAVE, lane = lane_id();
  int2* stk = s_stack + (size_t)wave * stack_depth * WAVE;
  const uint64_t below = lanes_below();
  const int xcd = blockIdx.x & 7;
  const int4* __restrict__ R = T.inode;
  const int32_t nint = (int32_t)(T.N - 1);
  for (int probe = 0; probe < 8; ++probe) {
    const int xr = (xcd + probe) & 7;
    const int r0 = xcd_range[xr], r1 = xcd_range[xr + 1];
    for (;;) {
      // every lane takes part in the fetch (lane 0 adds 1, the others 0), so
      // there is no lane-divergent region in the chunk loop
      const uint32_t t = atomicAdd(&xcd_ctr[xr], lane == 0 ? 1u : 0u);
      const int k = (int)__builtin_amdgcn_readfirstlane(t) + r0;
      if (k >= r1) break;
      int next = __builtin_amdgcn_readfirstlane(chunk_first[k]);
      const int end = __builtin_amdgcn_readfirstlane(chunk_end[k]);
      const int64_t cs = EMIT ? cell_start[chunk_pair[k]] : 0;
      uint32_t* const obase = EMIT ? out + 3 * chunk_off[k] : nullptr;
      uint64_t cursor = 0;
      bool has = false, overflow = false, runaway = false;
      int sp = 0;
      Rec RU{}, RV{};
      int32_t U = 0, V = 0;
      for (int64_t step = 0;; ++step) {
        if (step > step_cap) {  // beyond any chunk's possible work: give up, report
          runaway = true;
          break;
        }
        // acquire: stack first, then fresh items in lane order
        const bool want = !has;
        const uint64_t need = __ballot(want && sp == 0);
        const int avail = end - next;
        bool got = false, fresh = false;
        int2 q = make_int2(0, 0);
        if (want) {
          if (sp > 0) {
            --sp;
            q = stk[sp * WAVE + lane];
            got = true;
          } else {
            const int r = __popcll(need & below);
            if (r < avail) {
              q = items[next + r];
              got = fresh = true;
            }
          }
        }
        const int took = __popcll(need);
        next += took < avail ? took : (avail > 0 ? avail : 0);
        if (got) {
          U = q.x;
          V = q.y;
          RU = load_rec(R, U, nint);
          RV = load_rec(R, V, nint);
        }
        if (__ballot(has || got) == 0) break;
        bool e1 = false, e2 = false;
        u32x3 m1, m2;
        if (got) {
          has = true;
          if (fresh && separated(RU.box, RV.box, s)) {
            e1 = true;
            has = false;
            if (EMIT) m1 = make_emit(RU, RV, cs);
          }
        }
        if (has) {
          const bool splitU = box_diam(RU.box) > box_diam(RV.box);
          const Rec& P = splitU ? RU : RV;
          const int32_t c1 = rec_left(P), c2 = rec_right(P);
          const Rec C1 = load_rec(R, c1, nint), C2 = load_rec(R, c2, nint);
          const Rec O = splitU ? RV : RU;
          const bool s1 = separated(C1.box, O.box, s), s2 = separated(C2.box, O.box, s);
          if (EMIT) {
            if (s1) m1 = splitU ? make_emit(C1, O, cs) : make_emit(O, C1, cs);
            if (s2) m2 = splitU ? make_emit(C2, O, cs) : make_emit(O, C2, cs);
          }
          e1 = s1;
          e2 = s2;
          if (!s1 && !s2) {
            const int2 second = splitU ? make_int2(c2, V) : make_int2(U, c2);
            if (sp < stack_depth) {
              stk[sp * WAVE + lane] = second;
              ++sp;
            } else {
              overflow = true;
            }
          }
          if (!s1 || !s2) {
            const int32_t cn = !s1 ? c1 : c2;
            const Rec& CN = !s1 ? C1 : C2;
            if (splitU) {
              U = cn;
              RU = CN;
            } else {
              V = cn;
              RV = CN;
            }
          } else {
            has = false;
          }
        }
        const uint64_t b1 = __ballot(e1), b2 = __ballot(e2);
        if (EMIT) {
          // streaming (non-temporal) 12-byte stores: the output is written
          // once and must not evict the tree from L2
          const int n1 = __popcll(b1);
          if (e1) __builtin_nontemporal_store(m1, (u32x3_w*)(obase + 3 * (cursor + __popcll(b1 & below))));
          if (e2) __builtin_nontemporal_store(m2, (u32x3_w*)(obase + 3 * (cursor + n1 + __popcll(b2 & below))));
        }
        cursor += (uint64_t)(__popcll(b1) + __popcll(b2));
      }
      const bool bad = runaway || __ballot(overflow) != 0;
      if (bad) atomicOr(err, 1);
      if (!EMIT) chunk_cnt[k] = cursor;  // same value from every lane
    }
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

inline unsigned blocks(int64_t n, int bs = 256) { return (unsigned)(n > 0 ? ceil_div(n, bs) : 1); }

}  // namespace

#define LAUNCH(kern, n, ...) \
  do { if ((n) > 0) hipLaunchKernelGGL(kern, dim3(blocks(n)), dim3(256), 0, st, __VA_ARGS__); } while (0)

void launch_pack_nodes(const TreeView& T, int4* rec, hipStream_t st) { LAUNCH(k_pack_nodes, 2 * T.N - 1, T, rec); }
void launch_wspd_roots_flags(const TreeView& T, uint32_t* flag, hipStream_t st) { LAUNCH(k_roots_flags, T.N - 1, T, flag); }
void launch_wspd_roots_fill(const TreeView& T, const uint32_t* flag, const uint32_t* pos, int2* items, hipStream_t st) {
  LAUNCH(k_roots_fill, T.N - 1, T, flag, pos, items);
}
void launch_wspd_classify(const TreeView& T, const int2* items, int64_t f, int s, const WspdTuning& tun, uint64_t* cnt,
                          hipStream_t st) {
  LAUNCH(k_classify, f, T, items, f, s, tun.stack_depth, (int64_t)tun.work_cap, cnt);
}
void launch_wspd_scatter(const TreeView& T, const int2* items, int64_t f, const uint64_t* cnt, const uint64_t* pos,
                         int2* out_items, int64_t out_base, int2* next, hipStream_t st) {
  LAUNCH(k_scatter, f, T, items, f, cnt, pos, out_items, out_base, next);
}
void launch_item_keys(const TreeView& T, const int2* items, int64_t m, bool both, uint64_t* keys, hipStream_t st) {
  LAUNCH(k_item_keys, m, T, items, m, both ? 1 : 0, keys);
}
void launch_gather_items(const int2* src, const uint32_t* perm, int2* dst, int64_t m, hipStream_t st) {
  LAUNCH(k_gather_items, m, src, perm, dst, m);
}
void launch_item_bounds(const TreeView& T, const int2* items, int64_t m, int64_t* lo, int64_t* hi, hipStream_t st) {
  LAUNCH(k_item_bounds, m, T, items, m, lo, hi);
}
void launch_chunk_heads(const TreeView& T, const int2* items, int64_t m, const int64_t* item_start, int chunk,
                        uint32_t* head, hipStream_t st) {
  LAUNCH(k_chunk_heads, m, T, items, m, item_start, chunk, head);
}
void launch_chunk_fill(const TreeView& T, const int2* items, int64_t m, const int64_t* item_start,
                       const int32_t* items_per_pair, const uint32_t* head, const uint32_t* cid, int chunk,
                       int32_t* chunk_first, int32_t* chunk_end, int32_t* chunk_pair, hipStream_t st) {
  LAUNCH(k_chunk_fill, m, T, items, m, item_start, items_per_pair, head, cid, chunk, chunk_first, chunk_end, chunk_pair);
}
void launch_wspd_pass(bool emit, const TreeView& T, const int2* items, const int32_t* chunk_first,
                      const int32_t* chunk_end, const int32_t* chunk_pair, int64_t nchunks, const int32_t* xcd_range,
                      uint32_t* xcd_ctr, int s, const WspdTuning& tun, uint64_t* chunk_cnt, const uint64_t* chunk_off,
                      const int64_t* cell_start, uint32_t* out, int32_t* err, int num_cus, hipStream_t st) {
  if (nchunks <= 0) return;
  int64_t grid = (int64_t)num_cus * tun.blocks_per_cu;
  grid = ((grid + 7) / 8) * 8;
  const size_t lds = (size_t)4 * tun.stack_depth * WAVE * sizeof(int2);
  // A chunk's items each have at most work_cap leaf pairs, hence fewer than
  // 2 work_cap recursion nodes; every wave step resolves at least one.
  const int64_t step_cap = (int64_t)tun.chunk_items * (2 * (int64_t)tun.work_cap + 2) + 1024;
  if (emit)
    hipLaunchKernelGGL(k_wspd<true>, dim3((unsigned)grid), dim3(256), lds, st, T, items, chunk_first, chunk_end,
                       chunk_pair, xcd_range, xcd_ctr, s, tun.stack_depth, step_cap, chunk_cnt, chunk_off, cell_start, out, err);
  else
    hipLaunchKernelGGL(k_wspd<false>, dim3((unsigned)grid), dim3(256), lds, st, T, items, chunk_first, chunk_end,
                       chunk_pair, xcd_range, xcd_ctr, s, tun.stack_depth, step_cap, chunk_cnt, chunk_off, cell_start, out, err);
}
void launch_pair_totals(const uint64_t* chunk_cnt, const uint64_t* chunk_off, const int32_t* chunk_pair,
                        int64_t nchunks, uint64_t* pair_start, uint64_t* pair_end, uint64_t* npairs, int64_t K,
                        hipStream_t st) {
  LAUNCH(k_pair_bounds, nchunks, chunk_cnt, chunk_off, chunk_pair, nchunks, pair_start, pair_end);
  LAUNCH(k_pair_counts, K, pair_start, pair_end, K, npairs);
}

}  // namespace w1
