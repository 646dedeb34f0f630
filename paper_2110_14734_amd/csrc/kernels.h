// Host-side launchers of the stage kernels (internal).
#pragma once

#include "common.h"

namespace w1 {

// One input segment: the points of diagram `side` (0 = A, 1 = B) of pair
// `pair`, read from `ptr` and placed at packed index out_off.
struct SegDesc {
  const void* ptr;
  int64_t n;
  int64_t out_off;
  int32_t pair;
  int32_t side;
};

// a0
void launch_load(const SegDesc* segs, int nseg, int64_t total, int dtype, double* pb, double* pd, uint32_t* psd,
                 uint64_t* kw0, uint64_t* kw1, uint64_t* kw2, int32_t* perr, hipStream_t st);
void launch_group_heads(const uint32_t* perm, const uint64_t* kw2s, const double* pb, const double* pd, int64_t n,
                        uint32_t* head, hipStream_t st);
void launch_group_fill(const uint32_t* perm, const uint64_t* kw2s, const uint32_t* head, const uint32_t* gidx,
                       const double* pb, const double* pd, const uint32_t* psd, int64_t n, double* gb, double* gd,
                       uint32_t* gpair, int32_t* gw, hipStream_t st);
void launch_count_total(const uint32_t* head, const uint32_t* scanned, int64_t n, uint64_t* out, hipStream_t st);
// *out = scanned[n-1] + cnt[n-1] (total of an exclusive scan), 64-bit
void launch_count_total64(const uint64_t* cnt, const uint64_t* scanned, int64_t n, uint64_t* out, hipStream_t st);
void launch_nonzero_flags(const int32_t* gw, int64_t G, uint32_t* flag, hipStream_t st);
void launch_loc_fill(const int32_t* gw, const uint32_t* flag, const uint32_t* lidx, const double* gb, const double* gd,
                     const uint32_t* gpair, int64_t G, double* lb, double* ld, int32_t* lw, uint32_t* lpair,
                     const PairArrays& P, hipStream_t st);
// a1
void launch_loc_bbox(const double* lb, const double* ld, const uint32_t* lpair, int64_t M, const PairArrays& P,
                     hipStream_t st);
void launch_bucket_setup(const PairArrays& P, int64_t K, int64_t* nbuckets, hipStream_t st);
void launch_bucket_count(const double* lb, const double* ld, const int32_t* lw, const uint32_t* lpair, int64_t M,
                         const PairArrays& P, uint32_t* bincnt, int64_t* lbin, hipStream_t st);
void launch_bucket_fill(const double* lb, const double* ld, const int64_t* lbin, int64_t M, const uint32_t* binstart,
                        uint32_t* bincur, double2* ent, uint32_t* entl, hipStream_t st);
// RWMD nearest neighbours: every location starts at its diagonal cost, then
// one wave per bin (nbins = 2 * buckets + 1 bounds) searches the other side.
void launch_nn(const double* lb, const double* ld, const int32_t* lw, const uint32_t* lpair, int64_t M,
               const PairArrays& P, const uint32_t* binstart, const double2* ent, const uint32_t* entl, int64_t nbins,
               double* lt, double* lterm, bool l2, hipStream_t st);
void launch_term_max(const double* lterm, const int32_t* lw, const uint32_t* lpair, int64_t M, const PairArrays& P,
                     hipStream_t st);
void launch_rwmd_shift(const PairArrays& P, int64_t K, hipStream_t st);
void launch_term_sum(const double* lterm, const int32_t* lw, const uint32_t* lpair, int64_t M, const PairArrays& P,
                     hipStream_t st);
void launch_params(const PairArrays& P, int64_t K, double eps_c, bool l2, hipStream_t st);
// a2
void launch_snap(const double* lb, const double* ld, const uint32_t* lpair, int64_t M, const PairArrays& P, int64_t* li,
                 int64_t* lj, hipStream_t st);
void launch_morton(const int64_t* li, const int64_t* lj, const uint32_t* lpair, int64_t M, const PairArrays& P,
                   uint64_t* kw0, uint64_t* kw1, hipStream_t st);
void launch_cell_heads(const uint32_t* perm, const uint64_t* kw1s, const uint64_t* kw0, int64_t M, uint32_t* head,
                       hipStream_t st);
void launch_cell_fill(const uint32_t* perm, const uint64_t* kw1s, const uint64_t* kw0, const uint32_t* head,
                      const uint32_t* cidx, const int64_t* li, const int64_t* lj, const int32_t* lw, int64_t M,
                      const PairArrays& P, uint64_t* ckey, uint32_t* cpair, int2* cij, int32_t* ca, int32_t* cb,
                      hipStream_t st);
// pair-major runs: bounds of each pair's run, and their lengths
void launch_run_bounds(const uint32_t* key, int64_t n, int64_t* lo, int64_t* hi, hipStream_t st);
void launch_bounds_count32(const int64_t* lo, const int64_t* hi, int64_t K, int32_t* out, hipStream_t st);
// a3
void launch_karras(const uint32_t* cpair, const uint64_t* ckey, int64_t N, int4* iaux, int32_t* iparent,
                   hipStream_t st);
// Depth of each internal node (maxd: the largest; zero it first), then the
// tight boxes and heights one depth level per launch, deepest first.
void launch_node_depth(const int32_t* iparent, int64_t N, int32_t* depth, int32_t* maxd, hipStream_t st);
void launch_level_boxes(const int2* cij, int64_t N, const int4* iaux, const int32_t* depth, int d, int4* ibox,
                        int32_t* iheight, hipStream_t st);

// a5: the network in compressed sparse row form (csr.hip).  Geometry
// (csr_geometry in limits.h): a bucket is 2^RB consecutive cells, heads take
// DB bits, RB + DB <= 32, at most 1024 buckets.
int csr_bucket_stride();
size_t csr_bucket_scatter_lds(int NB);
size_t csr_row_scatter_lds(int RB);
int64_t csr_entry_tile(int RB);  // entries per tile of the row scatter
int64_t csr_hist_tile(int RB);   // entries per tile of the row histogram
// Records per tile of the bucket scatter: a block of the blocked emission
// holds at most this many.
int csr_tile_records();
void launch_csr_bucket_scatter(const uint32_t* rec, int rec_words, uint64_t P, const uint64_t* rstart, int64_t K,
                               const int64_t* cell_start, int RB, int DB, int NB, const uint64_t* bstart,
                               uint64_t* bcur, uint32_t* out,
                               const uint32_t* blk_fill, const uint32_t* blk_pair, uint32_t blk_recs,
                               uint32_t nblocks, hipStream_t st);
void launch_csr_row_hist(const uint32_t* ent, const int64_t* tfirst, int64_t ntiles, int NB, const uint64_t* bstart,
                         int RB, int DB, int64_t N, uint32_t* rowcnt, hipStream_t st);
void launch_csr_bflags(const int32_t* cb, int64_t N, uint32_t* flag, hipStream_t st);
void launch_csr_row_deg(const uint32_t* cpair, const int64_t* cell_start, const int32_t* ncells, const int32_t* ca,
                        const int32_t* cb, const uint32_t* rowcnt, const uint32_t* bpos, int64_t N, uint64_t* deg,
                        hipStream_t st);
void launch_csr_row_scatter(const uint32_t* ent, const int64_t* tfirst, int64_t ntiles, int NB,
                            const uint64_t* bstart, int RB, int DB, int64_t N, const uint32_t* cpair,
                            const uint64_t* off, uint32_t* rowcur, uint32_t* heads, hipStream_t st);
void launch_csr_row_sort(const uint32_t* cpair, const int64_t* cell_start, const int32_t* ncells, const int2* cij,
                         const int32_t* ca, const uint32_t* rowcnt, const uint64_t* off, const uint32_t* heads,
                         int64_t N, int64_t max_pair_cells, int window_words, int num_cus, const int32_t* costK, uint32_t* col,
                         void* cost, uint64_t* rowq /* row queue counter, zero at launch */, hipStream_t st);
void launch_csr_bdiag(const uint32_t* cpair, const int64_t* cell_start, const int32_t* ncells, const int2* cij,
                      const int32_t* ca, const int32_t* cb, const uint32_t* bpos, const uint64_t* off,
                      const PairArrays& P, int64_t N, const int32_t* costK, uint32_t* col, void* cost,
                      int64_t* supply, hipStream_t st);
// Euclidean network: costs int64 in units of g 2^-costK[pair] (costK NULL:
// L-infinity int32 costs).  Largest shifted cell coordinate per pair:
void launch_pair_xmax(const uint32_t* cpair, const int2* cij, int64_t N, uint64_t* xmax, hipStream_t st);
void launch_csr_local_rowptr(const uint32_t* cpair, const int64_t* cell_start, const int32_t* ncells,
                             const uint64_t* off, int64_t N, int64_t* rp, hipStream_t st);
// out[p] = off[cell_start[p] + 2p] for p < K, out[K] = off[nrows]: each pair's
// first arc and the arc total.
void launch_csr_pair_arcs(const int64_t* cell_start, const uint64_t* off, int64_t K, int64_t nrows, uint64_t* out,
                          hipStream_t st);

// a4 ------------------------------------------------------------------------
// Tree view used by the WSPD traversal.  Node reference r >= 0 is internal
// node r, r < 0 is the leaf of cell ~r.
struct TreeView {
  const int4* inode;    // traversal records, 2 int4 each, 2N - 1 of them:
                        // root first, siblings adjacent (see k_pack_nodes)
  const int4* ibox;     // internal: min_i, min_j, max_i, max_j
  const int4* iaux;     // internal: left, right, lo, hi
  const int32_t* iheight;
  const int2* cij;      // cell coordinates
  const uint32_t* cpair;
  int64_t N;
};

// Tail-bucket histogram of the network's arcs, taken by the emit pass:
// bucket of a global cell c = c >> RB, NB buckets (NB = 0: none).  Records
// hold cells local to their diagram pair, whose first cell is
// cell_start[chunk_pair[chunk]].
struct BucketHist {
  const int32_t* chunk_pair = nullptr;
  const int64_t* cell_start = nullptr;
  int RB = 0, NB = 0;
  uint64_t* count = nullptr;
};

// Emit pass output placement: records of chunk k start at word
// 3 (chunk_off[k] - base) of the output; with chunk_sum set, the pass also
// writes each chunk's record checksum (sum h, sum h^2) to chunk_sum[2k..].
struct StreamOut {
  int64_t base = 0;                   // first pair of the arena fill (if base_dev is null)
  const int64_t* base_dev = nullptr;  // device copy of it, read at launch (graph replays)
  uint64_t* chunk_sum = nullptr;
  int64_t slot = 0;  // > 0: chunk k writes its records at k * slot (and its count), no count pass needed
};

// Emit pass output in blocks, for the network path (no count pass; the
// records carry no cost, which the network takes from the cells): each
// wave takes blocks of `block` records from a global counter as it fills
// them, and a block holds the records of one diagram pair.  When a block is
// full or the wave moves to another pair, fill[b] and pair[b] describe it and
// its records are added to pair_count[pair].  A wave that finds no block left
// sets *overflow and writes no more records (the caller then falls back to
// the counted layout).
struct BlockOut {
  uint32_t* base = nullptr;  // max_blocks * block records of (u, v), 8 bytes each
  uint32_t block = 0;        // records per block (2 * WAVE <= block)
  uint32_t max_blocks = 0;
  uint32_t* nblocks = nullptr;
  uint32_t* fill = nullptr;
  uint32_t* pair = nullptr;
  unsigned long long* pair_count = nullptr;
  int32_t* overflow = nullptr;
  const int32_t* chunk_pair = nullptr;
};

struct WspdTuning {
  int stack_depth;  // per-lane DFS stack entries (LDS), items need height sum < this
  int work_cap;     // items need |U| * |V| <= cap to skip the expansion rounds; this is the
                    // largest cap, small diagram pairs use smaller ones
  int chunk_items;  // items per chunk of the count / emit passes
  int blocks_per_cu;
  int compact;      // 1: packed split records when coordinates allow, 0: never
};

// Traversal records (2N - 1 of them) and rmap: node reference -> record
// (internal node r -> rmap[r], cell c -> rmap[N - 1 + c]).
void launch_pack_nodes(const TreeView& T, const int64_t* cell_start, int4* rec, int32_t* rmap, hipStream_t st);
// Packed split records (N - 1 of them, 2 uint4 each); every cell coordinate
// must be below 2^28.
void launch_pack_split(const TreeView& T, uint4* out, hipStream_t st);
// Final work items (node references) -> work entries of the passes.
void launch_item_prep(const TreeView& T, const int2* items, const uint32_t* perm, int64_t m, int s, const int32_t* rmap, bool l2,
                      int2* out, hipStream_t st);
void launch_wspd_roots_flags(const TreeView& T, uint32_t* flag, hipStream_t st);
void launch_wspd_roots_fill(const TreeView& T, const uint32_t* flag, const uint32_t* pos, int2* items, hipStream_t st);
// pair_cap[p]: the work cap of diagram pair p (at most tun.work_cap).
void launch_wspd_classify(const TreeView& T, const int2* items, int64_t f, int s, const WspdTuning& tun,
                          const int32_t* pair_cap, bool prune, bool l2, uint64_t* cnt, hipStream_t st);
void launch_wspd_scatter(const TreeView& T, const int2* items, int64_t f, const uint64_t* cnt, const uint64_t* pos,
                         int2* out_items, int64_t out_base, bool l2, int2* next, hipStream_t st);
// All expansion rounds of a small work list in one workgroup, starting from
// the f0 items at `roots` (left unchanged): kept items go to kept[0, ctl[0]),
// the frontiers alternate between fa and fb (cap_front items each).
// ctl[1] = 0 done, 1 out of room (nothing usable), 2 more than max_rounds
// rounds.  The work list equals the round-by-round one.
void launch_wspd_expand_small(const TreeView& T, const int2* roots, int64_t f0, int s, const WspdTuning& tun,
                              const int32_t* pair_cap, bool prune, bool l2, int max_rounds, int2* kept,
                              int64_t cap_kept, int2* fa, int2* fb, int64_t cap_front, int64_t* ctl, hipStream_t st);
void launch_item_keys(const TreeView& T, const int2* items, int64_t m, bool both, uint64_t* keys, hipStream_t st);
void launch_gather_items(const int2* src, const uint32_t* perm, int2* dst, int64_t m, hipStream_t st);
// Per-pair item runs of the sorted work list (keys: first representative
// cells), and the chunks from the per-pair item counts: cstart[p] = first
// chunk of pair p (K + 1 values, cstart[K] = nch).
void launch_item_bounds(const uint32_t* cpair, const uint64_t* keys, int64_t m, int64_t* lo, int64_t* hi,
                        hipStream_t st);
void launch_chunks(const int32_t* cstart, int64_t K, const int64_t* item_start, const int32_t* ipp, int64_t nch,
                   int chunk, int32_t* chunk_first, int32_t* chunk_end, int32_t* chunk_pair, hipStream_t st);
// Count (emit = false) or emit pass; split_recs = packed split records, or
// nullptr to read the children's records.  An emit pass uses the packed
// records only for the network's records (a bucket histogram, no checksums,
// no blocks), which are then (u, v) pairs.  Returns the words per record
// written: 0 (count pass), 2 (u, v) or 3 (u, v, cost).
int launch_wspd_pass(bool emit, const TreeView& T, const uint4* split_recs, const int2* items,
                      const int32_t* chunk_first, const int32_t* chunk_end, int64_t nchunks, const int32_t* xcd_range,
                      uint32_t* xcd_ctr, int s, const WspdTuning& tun, uint64_t* chunk_cnt, const uint64_t* chunk_off,
                      uint32_t* out, int32_t* err, bool prune, bool l2, const BucketHist& bh, const StreamOut& so,
                      const BlockOut& bo, int chunk_stride,
                      int num_cus, hipStream_t st);
// Streamed emission: next arena fill of a replayed launch sequence.  Fill
// r = *ctr (of nruns) copies its chunk ranges per XCD (9 values at
// run_xr + 9 r) into xr and its first pair into *base, clears the 8 chunk
// counters xc and advances *ctr; past the last fill, the ranges are empty.
void launch_stream_next(const int32_t* run_xr, const int64_t* run_base, int nruns, int32_t* ctr, int32_t* xr,
                        int64_t* base, uint32_t* xc, hipStream_t st);
// Records of slotted chunks (cnt[k] records of w words at k * slot) moved
// to their scanned offsets off[k].
void launch_compact_slots(const uint32_t* src, const uint64_t* cnt, const uint64_t* off, int64_t nch, int64_t slot,
                          int w, uint32_t* dst, hipStream_t st);
void launch_pair_totals(const uint64_t* chunk_cnt, const uint64_t* chunk_off, const int32_t* chunk_pair,
                        int64_t nchunks, uint64_t* pair_start, uint64_t* pair_end, uint64_t* npairs, int64_t K,
                        hipStream_t st);

}  // namespace w1
