// Host orchestration of the approximate W1 pipeline and the C-ABI entry
// points declared in include/w1approx.h.
//
// Stage order (Alg. 3): a0 0-condensation, a1 RWMD, a2 grid condensation,
// a3 radix tree, a4 WSPD pairs, a5 diagonal arcs and supplies, then the host
// network simplex.  A batch of k pairs runs every stage once over all pairs;
// a single pair is a batch of one.  The host reads back a few counts between
// stages to size buffers; everything else stays on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "../../include/w1approx.h"
#include "common.h"
#include "ctx.h"
#include "flow.h"
#include "kernels.h"
#include "limits.h"

namespace w1 {

namespace {

inline int clz64(uint64_t x) { return x ? __builtin_clzll(x) : 64; }
inline int bitlen_u64(uint64_t x) { return 64 - clz64(x); }
inline int ctz64(uint64_t x) { return x ? __builtin_ctzll(x) : 64; }

constexpr int kSortMaxWords = 3;
// Largest launch group (in cells) whose work list may be expanded in one
// workgroup (k_expand_small) rather than round by round.
constexpr int32_t kFusedExpandMaxCells = 65536;

// Stable sort of n elements by the words (least significant first); returns
// the permutation in *perm and the sorted most significant word in *top.
void sort_words(Ctx& c, const uint64_t* const* words, int nw, int64_t n, uint32_t** perm, uint64_t** top) {
  uint64_t* kA = need<uint64_t>(c, c.kA, n);
  uint64_t* kB = need<uint64_t>(c, c.kB, n);
  uint32_t* vA = need<uint32_t>(c, c.vA, n);
  uint32_t* vB = need<uint32_t>(c, c.vB, n);
  void* tmp = need<char>(c, c.sorttmp, (int64_t)radix_tmp_bytes(n));
  // the bits that vary in each word (OR ^ AND over its elements): reordering
  // a word does not change them, so one read-back serves every word
  if (nw > kSortMaxWords) throw StageError{W1_EINVAL};
  uint64_t* orand = need<uint64_t>(c, c.small, 64) + 8;
  uint64_t* part = need<uint64_t>(c, c.orpart, 2 * kOrAndBlocks);
  for (int w = 0; w < nw; ++w) key_or_and(words[w], n, orand + 2 * w, part, c.st);
  readback(c, orand, c.hpin, 2 * nw);
  uint64_t vary[kSortMaxWords];
  for (int w = 0; w < nw; ++w) vary[w] = c.hpin[2 * w] ^ c.hpin[2 * w + 1];
  iota_u32(vA, n, c.st);
  for (int w = 0; w < nw; ++w) {
    if (!vary[w] && w + 1 < nw) continue;  // the last word is returned sorted, so always taken
    if (w == 0) check(c, hipMemcpyAsync(kA, words[0], (size_t)n * 8, hipMemcpyDeviceToDevice, c.st));
    else gather_u64(words[w], vA, kA, n, c.st);
    if (!vary[w]) continue;
    const int lo = ctz64(vary[w]), hi = 64 - clz64(vary[w]);
    if (radix_sort(kA, vA, kB, vB, n, lo, hi, tmp, c.st)) {
      std::swap(kA, kB);
      std::swap(vA, vB);
      std::swap(c.kA, c.kB);
      std::swap(c.vA, c.vB);
    }
  }
  *perm = vA;
  *top = kA;
}

uint32_t* scan_flags(Ctx& c, const uint32_t* flags, int64_t n, DBuf& out) {
  uint32_t* o = need<uint32_t>(c, out, n);
  scan_u32(flags, o, n, need<char>(c, c.scantmp, (int64_t)scan_tmp_bytes(n, 8)), c.st);
  return o;
}

uint64_t total_of(Ctx& c, const uint32_t* flags, const uint32_t* scanned, int64_t n) {
  if (n <= 0) return 0;
  uint64_t* slot = need<uint64_t>(c, c.small, 64);
  launch_count_total(flags, scanned, n, slot, c.st);
  return read_u64(c, slot);
}

struct Opts {
  double eps = 0.1, kappa = 0.1;
  int s = 0;
  uint32_t flags = 0;
  int64_t pivot_cap = 0;
};

int separation(double eps, double kappa) {
  const double ec = kappa * eps;
  const double tau = (eps - 2.0 * ec) / (1.0 + ec);
  int s = (int)std::ceil(2.0 + 4.0 / tau);
  if (s < 3) s = 3;
  for (;;) {
    const double t = (double)(s + 2) / (double)(s - 2);
    if (t + (t + 1.0) * ec <= 1.0 + eps) break;
    ++s;
  }
  return s;
}

void setup_pairs(Ctx& c, int64_t K) {
  // 26 int64-sized and 14 int32-sized slots per pair (some spare), all in
  // one allocation, so the results come back in one transfer
  const int64_t K8 = ((K + 31) / 32) * 32;
  c.pair_bytes = K8 * 8 * 26 + K8 * 4 * 14;
  char* base = need<char>(c, c.pairs, c.pair_bytes);
  int64_t off = 0;
  auto take8 = [&](void) { void* p = base + off; off += K8 * 8; return p; };
  auto take4 = [&](void) { void* p = base + off; off += K8 * 4; return p; };
  PairArrays& P = c.P;
  P.nA = (int64_t*)take8(); P.nB = (int64_t*)take8(); P.loc_start = (int64_t*)take8();
  P.bmax = (uint64_t*)take8(); P.dmax = (uint64_t*)take8(); P.bx0 = (int64_t*)take8(); P.by0 = (int64_t*)take8();
  P.bbase = (int64_t*)take8(); P.tmaxA = (uint64_t*)take8(); P.tmaxB = (uint64_t*)take8();
  P.sumA = (uint64_t*)take8(); P.sumB = (uint64_t*)take8(); P.L = (double*)take8();
  P.cell_start = (int64_t*)take8(); P.item_start = (int64_t*)take8(); P.npairs = (uint64_t*)take8();
  P.pair_start = (uint64_t*)take8(); off += K8 * 8;  // spare
  const int64_t zero8_end = off;
  P.bmin = (uint64_t*)take8(); P.dmin = (uint64_t*)take8(); P.m0 = (int64_t*)take8();
  const int64_t ones8_end = off;
  P.seg_lo = (int64_t*)take8(); P.seg_hi = (int64_t*)take8();
  off += K8 * 8;  // spare
  P.err = (int32_t*)take4(); P.locA = (int32_t*)take4(); P.locB = (int32_t*)take4(); P.beh = (int32_t*)take4();
  P.bnx = (int32_t*)take4(); P.bny = (int32_t*)take4(); P.FA = (int32_t*)take4(); P.FB = (int32_t*)take4();
  P.e = (int32_t*)take4(); P.ncells = (int32_t*)take4(); P.costK = (int32_t*)take4();
  fill_u64((uint64_t*)base, 0, zero8_end / 8, c.st);
  fill_u64((uint64_t*)P.bmin, ~0ull, K8 * 2, c.st);
  fill_u64((uint64_t*)P.m0, (uint64_t)INT64_MAX, K8, c.st);
  (void)ones8_end;
  fill_u32((uint32_t*)P.err, 0, K8 * 11, c.st);
}

template <typename T>
std::vector<T> fetch_pairs(Ctx& c, const T* dev, int64_t K) {
  std::vector<T> h((size_t)K);
  readback(c, dev, h.data(), K);
  return h;
}

// The per-pair array `dev` out of a host copy of the whole per-pair block.
template <typename T>
std::vector<T> from_pair_block(const Ctx& c, const std::vector<char>& block, const T* dev, int64_t K) {
  const T* x = (const T*)(block.data() + ((const char*)dev - (const char*)c.pairs.p));
  return std::vector<T>(x, x + K);
}

void record(Ctx& c, int i) {
  check(c, hipEventRecord(c.ev[i], c.st));
  if (c.trace) {
    static const char* names[] = {"start", "a0 condense0", "a1 rwmd", "a2 grid", "a3 tree", "a4 wspd", "a5 arcs", "end"};
    check(c, hipStreamSynchronize(c.st));
    std::fprintf(stderr, "[w1] %s done\n", names[i]);
    std::fflush(stderr);
  }
}

void trace(Ctx& c, const char* what, int64_t v) {
  if (!c.trace) return;
  std::fprintf(stderr, "[w1]   %s = %lld\n", what, (long long)v);
  std::fflush(stderr);
}

// Work cap of one diagram pair.  A pair of n cells has about n^2 / 2 leaf
// pairs; at the tuned cap a small pair forms a few thousand items of up to
// cap leaf pairs each, which fill only a handful of chunks, so a handful of
// waves would run its whole traversal.  Such a pair (n^2 / 2 below 2^14
// times the tuned cap) gets the largest power of two c >= 16 with
// 2^14 c <= n^2 / 2, else 16.  The cap depends on the pair alone, so its
// output order is the same alone and in a batch.
int pair_work_cap(int64_t ncells, int tuned) {
  const double leaf_pairs = 0.5 * (double)ncells * (double)ncells;
  if (leaf_pairs >= 16384.0 * tuned) return tuned;
  int cap = 16;
  while (2.0 * cap * 16384.0 <= leaf_pairs) cap *= 2;
  return std::min(cap, tuned);
}

// A captured launch sequence: released (after the stream it was replayed
// on has drained) when the guard goes out of scope, also on an error.
struct GraphGuard {
  hipStream_t cap = nullptr, wait = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool capturing = false;
  ~GraphGuard() {
    if (capturing) {
      hipGraph_t g = nullptr;
      (void)hipStreamEndCapture(cap, &g);
      if (g) (void)hipGraphDestroy(g);
    }
    if (exec && wait) (void)hipStreamSynchronize(wait);
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cap) (void)hipStreamDestroy(cap);
  }
};

// ------------------------------------------------------------------ pipeline --
int run(Ctx& c, const w1_pd* a, const w1_pd* b, int64_t K, const Opts& o, hipStream_t st, w1_result* res,
        double* L_only) {
  c.st = st;
  c.network_valid = false;
  c.K = K;
  int dtype = -1;
  int64_t total = 0;
  const bool dev_in = (o.flags & W1_INPUT_DEVICE) != 0;
  for (int64_t p = 0; p < K; ++p) {
    for (int side = 0; side < 2; ++side) {
      const w1_pd& d = side ? b[p] : a[p];
      if (d.n < 0 || (d.n > 0 && !d.xy) || (d.dtype != W1_F32 && d.dtype != W1_F64) || d.reserved != 0) return W1_EINVAL;
      if (dtype < 0) dtype = d.dtype;
      if (d.dtype != dtype) return W1_EINVAL;
      total += d.n;
    }
  }
  if (total >= (int64_t(1) << 31) || K >= (int64_t(1) << 30)) return W1_EINVAL;
  const int s = o.s > 0 ? o.s : separation(o.eps, o.kappa);
  const bool prune = (o.flags & W1_PRUNE) != 0;
  const bool l2 = (o.flags & W1_METRIC_L2) != 0;
  if (l2 && prune) return W1_EINVAL;  // pruning is exact for the integer L-infinity costs only
  // condensation share of the error: kappa * eps, or the paper's own choice
  // for a given sparsity parameter (Alg. 2, Alg. 3)
  double eps_c = o.kappa * o.eps;
  if (o.flags & W1_PAPER_GRID) {
    if (o.s <= 0) return W1_EINVAL;
    eps_c = o.s >= 12 ? 8.0 / (double)(o.s - 4) : 1.0;
  }
  for (int i = 0; i < 8; ++i) record(c, i);
  record(c, 0);

  // ---------------------------------------------------------------- a0 --
  const size_t esz = dtype == W1_F32 ? 4 : 8;
  // input segments; an allocation-free call uses the context's fixed table
  std::vector<SegDesc> seg_vec;
  SegDesc* segs = c.seg_fixed;
  if (!c.arena.base) {
    seg_vec.resize((size_t)(2 * K));
    segs = seg_vec.data();
  } else if (K > kNoAllocMaxPairs) {
    return W1_ERANGE;
  }
  int64_t nseg = 0;
  char* staging = nullptr;
  if (!dev_in && total > 0) staging = need<char>(c, c.stage, total * 2 * (int64_t)esz);
  int64_t off = 0;
  for (int64_t p = 0; p < K; ++p)
    for (int side = 0; side < 2; ++side) {
      const w1_pd& d = side ? b[p] : a[p];
      if (d.n == 0) continue;
      const void* ptr = d.xy;
      if (!dev_in) {
        check(c, hipMemcpyAsync(staging + off * 2 * esz, d.xy, (size_t)d.n * 2 * esz, hipMemcpyHostToDevice, st));
        ptr = staging + off * 2 * esz;
      }
      segs[nseg++] = SegDesc{ptr, d.n, off, (int32_t)p, side};
      off += d.n;
    }
  setup_pairs(c, K);
  PairArrays& P = c.P;
  int64_t M = 0, N = 0;
  if (total > 0) {
    SegDesc* dsegs = need<SegDesc>(c, c.segs, nseg);
    upload(c, dsegs, segs, (size_t)nseg * sizeof(SegDesc));
    double* pb = need<double>(c, c.pb, total);
    double* pd = need<double>(c, c.pd, total);
    uint32_t* psd = need<uint32_t>(c, c.psd, total);
    uint64_t* kw0 = need<uint64_t>(c, c.kw0, total);
    uint64_t* kw1 = need<uint64_t>(c, c.kw1, total);
    uint64_t* kw2 = need<uint64_t>(c, c.kw2, total);
    launch_load(dsegs, (int)nseg, total, dtype, pb, pd, psd, kw0, kw1, kw2, P.err, st);
    check(c, hipGetLastError());
    uint32_t* perm;
    uint64_t* kw2s;
    const uint64_t* words[3] = {kw0, kw1, kw2};
    sort_words(c, words, 3, total, &perm, &kw2s);
    uint32_t* head = need<uint32_t>(c, c.head, total);
    launch_group_heads(perm, kw2s, pb, pd, total, head, st);
    uint32_t* gidx = scan_flags(c, head, total, c.idx);
    const int64_t G = (int64_t)total_of(c, head, gidx, total);
    trace(c, "points", total);
    trace(c, "groups", G);
    double* gb = need<double>(c, c.gb, G);
    double* gd = need<double>(c, c.gd, G);
    uint32_t* gpair = need<uint32_t>(c, c.gpair, G);
    int32_t* gw = need<int32_t>(c, c.gw, G);
    fill_u32((uint32_t*)gw, 0, G, st);
    launch_group_fill(perm, kw2s, head, gidx, pb, pd, psd, total, gb, gd, gpair, gw, st);
    uint32_t* flag = need<uint32_t>(c, c.head, G);
    launch_nonzero_flags(gw, G, flag, st);
    uint32_t* lidx = scan_flags(c, flag, G, c.idx);
    M = (int64_t)total_of(c, flag, lidx, G);
    trace(c, "locations", M);
    double* lb = need<double>(c, c.lb, M);
    double* ld = need<double>(c, c.ld, M);
    int32_t* lw = need<int32_t>(c, c.lw, M);
    uint32_t* lpair = need<uint32_t>(c, c.lpair, M);
    launch_loc_fill(gw, flag, lidx, gb, gd, gpair, G, lb, ld, lw, lpair, P, st);
    check(c, hipGetLastError());
  }
  record(c, 1);

  // ---------------------------------------------------------------- a1 --
  if (M > 0) {
    const double* lb = (const double*)c.lb.p;
    const double* ld = (const double*)c.ld.p;
    const int32_t* lw = (const int32_t*)c.lw.p;
    const uint32_t* lpair = (const uint32_t*)c.lpair.p;
    launch_loc_bbox(lb, ld, lpair, M, P, st);
    int64_t* nbk = need<int64_t>(c, c.nbuck, K + 1);
    launch_bucket_setup(P, K, nbk, st);
    scan_i64(nbk, P.bbase, K, need<char>(c, c.scantmp, (int64_t)scan_tmp_bytes(K, 8)), st);
    // the last pair's first bucket and bucket count, one wait for both
    check(c, hipMemcpyAsync(c.hpin, P.bbase + (K - 1), 8, hipMemcpyDeviceToHost, st));
    check(c, hipMemcpyAsync(c.hpin + 1, nbk + (K - 1), 8, hipMemcpyDeviceToHost, st));
    check(c, hipStreamSynchronize(st));
    const int64_t Btot = (int64_t)c.hpin[0] + (int64_t)c.hpin[1];
    trace(c, "rwmd buckets", Btot);
    const int64_t nbins = 2 * Btot + 1;
    if (nbins >= (int64_t(1) << 31)) throw StageError{W1_ERANGE};  // one workgroup per bin in the NN search
    uint32_t* bincnt = need<uint32_t>(c, c.bincnt, nbins);
    fill_u32(bincnt, 0, nbins, st);
    int64_t* lbin = need<int64_t>(c, c.lbin, M);
    launch_bucket_count(lb, ld, lw, lpair, M, P, bincnt, lbin, st);
    uint32_t* binstart = need<uint32_t>(c, c.binstart, nbins);
    scan_u32(bincnt, binstart, nbins, need<char>(c, c.scantmp, (int64_t)scan_tmp_bytes(nbins, 8)), st);
    fill_u32(bincnt, 0, nbins, st);
    double2* ent = need<double2>(c, c.ent, M);
    uint32_t* entl = need<uint32_t>(c, c.entl, M);
    launch_bucket_fill(lb, ld, lbin, M, binstart, bincnt, ent, entl, st);
    double* lt = need<double>(c, c.lt, M);
    double* lterm = need<double>(c, c.lterm, M);
    launch_nn(lb, ld, lw, lpair, M, P, binstart, ent, entl, nbins, lt, lterm, l2, st);
    launch_term_max(lterm, lw, lpair, M, P, st);
    launch_rwmd_shift(P, K, st);
    launch_term_sum(lterm, lw, lpair, M, P, st);
    launch_params(P, K, eps_c, l2, st);
    check(c, hipGetLastError());
  }
  record(c, 2);
  if (L_only) {  // straight into the caller's array, no host buffers
    int32_t* er = c.err_fixed;
    std::vector<int32_t> er_vec;
    if (K > kNoAllocMaxPairs) {
      er_vec.resize((size_t)K);
      er = er_vec.data();
    }
    check(c, hipMemcpyAsync(L_only, P.L, (size_t)K * 8, hipMemcpyDeviceToHost, st));
    check(c, hipMemcpyAsync(er, P.err, (size_t)K * 4, hipMemcpyDeviceToHost, st));
    check(c, hipStreamSynchronize(st));
    for (int64_t p = 0; p < K; ++p)
      if (er[p] == -1) L_only[p] = NAN;
    return W1_OK;
  }

  // ---------------------------------------------------------------- a2 --
  int64_t maxnp = 0;  // most cells of one diagram pair
  int32_t maxcap = 0;  // largest per-pair work cap of the launch group
  if (M > 0) {
    const double* lb = (const double*)c.lb.p;
    const double* ld = (const double*)c.ld.p;
    const int32_t* lw = (const int32_t*)c.lw.p;
    const uint32_t* lpair = (const uint32_t*)c.lpair.p;
    int64_t* li = need<int64_t>(c, c.li, M);
    int64_t* lj = need<int64_t>(c, c.lj, M);
    launch_snap(lb, ld, lpair, M, P, li, lj, st);
    uint64_t* kw0 = need<uint64_t>(c, c.kw0, M);
    uint64_t* kw1 = need<uint64_t>(c, c.kw1, M);
    launch_morton(li, lj, lpair, M, P, kw0, kw1, st);
    uint32_t* perm;
    uint64_t* kw1s;
    const uint64_t* words[2] = {kw0, kw1};
    sort_words(c, words, 2, M, &perm, &kw1s);
    uint32_t* head = need<uint32_t>(c, c.head, M);
    launch_cell_heads(perm, kw1s, kw0, M, head, st);
    uint32_t* cidx = scan_flags(c, head, M, c.idx);
    N = (int64_t)total_of(c, head, cidx, M);
    trace(c, "cells", N);
    uint64_t* ckey = need<uint64_t>(c, c.ckey, N);
    uint32_t* cpair = need<uint32_t>(c, c.cpair, N);
    int2* cij = need<int2>(c, c.cij, N);
    int32_t* ca = need<int32_t>(c, c.ca, N);
    int32_t* cb = need<int32_t>(c, c.cb, N);
    fill_u32((uint32_t*)ca, 0, N, st);
    fill_u32((uint32_t*)cb, 0, N, st);
    launch_cell_fill(perm, kw1s, kw0, head, cidx, li, lj, lw, M, P, ckey, cpair, cij, ca, cb, st);
    fill_u64((uint64_t*)P.seg_lo, 0, K, st);
    fill_u64((uint64_t*)P.seg_hi, 0, K, st);
    launch_run_bounds(cpair, N, P.seg_lo, P.seg_hi, st);
    launch_bounds_count32(P.seg_lo, P.seg_hi, K, P.ncells, st);
    // cell_start = exclusive scan of ncells (int32 -> int64 via host, K is small)
    std::vector<int32_t> nc = fetch_pairs(c, P.ncells, K);
    std::vector<int64_t> cs((size_t)K);
    int64_t acc = 0;
    for (int64_t p = 0; p < K; ++p) {
      cs[(size_t)p] = acc;
      acc += nc[(size_t)p];
      maxnp = std::max<int64_t>(maxnp, nc[(size_t)p]);
    }
    std::vector<int32_t> cap((size_t)K);
    for (int64_t p = 0; p < K; ++p) {
      cap[(size_t)p] = pair_work_cap(nc[(size_t)p], c.tun.work_cap);
      maxcap = std::max(maxcap, cap[(size_t)p]);
    }
    upload_all(c, {{P.cell_start, cs.data(), (size_t)K * 8}, {need<int32_t>(c, c.pcap, K), cap.data(), (size_t)K * 4}});
    check(c, hipGetLastError());
  }
  record(c, 3);

  // ---------------------------------------------------------------- a3 --
  TreeView T{};
  const uint4* split = nullptr;
  if (N > 0) {
    T.cij = (const int2*)c.cij.p;
    T.cpair = (const uint32_t*)c.cpair.p;
    T.N = N;
  }
  if (N >= 2) {
    int4* iaux = need<int4>(c, c.iaux, N - 1);
    int4* ibox = need<int4>(c, c.ibox, N - 1);
    int32_t* ih = need<int32_t>(c, c.iheight, N - 1);
    int32_t* ipar = need<int32_t>(c, c.iparent, N - 1);
    int32_t* depth = need<int32_t>(c, c.ndepth, N - 1);
    launch_karras((const uint32_t*)c.cpair.p, (const uint64_t*)c.ckey.p, N, iaux, ipar, st);
    int32_t* dmax_d = (int32_t*)need<uint64_t>(c, c.small, 64);
    fill_u32((uint32_t*)dmax_d, 0, 1, st);
    launch_node_depth(ipar, N, depth, dmax_d, st);
    int32_t dmax = 0;
    readback(c, dmax_d, &dmax, 1);
    if (dmax >= N - 1) throw StageError{W1_EOVERFLOW};  // a parent chain longer than the tree
    for (int d = dmax; d >= 0; --d) launch_level_boxes((const int2*)c.cij.p, N, iaux, depth, d, ibox, ih, st);
    T.ibox = ibox;
    T.iaux = iaux;
    T.iheight = ih;
    if (N >= (int64_t(1) << 30)) throw StageError{W1_ERANGE};  // work entries hold record numbers in 31 bits
    // one leading pad record: sibling pairs (records 2g + 1, 2g + 2) then
    // start on 64-byte boundaries and never straddle a cache line
    int4* inode = need<int4>(c, c.inode, 2 * (2 * N)) + 2;
    launch_pack_nodes(T, P.cell_start, inode, need<int32_t>(c, c.rmap, 2 * N - 1), st);
    T.inode = inode;
    if (c.tun.compact) {  // the root's box bounds every coordinate (all are >= 0)
      int4 root;
      readback(c, ibox, &root, 1);
      if (std::max(root.z, root.w) < (1 << 28)) {
        uint4* sr = need<uint4>(c, c.isplit, 2 * (N - 1));
        launch_pack_split(T, sr, st);
        split = sr;
      }
    }
    trace(c, "packed split records", split ? 1 : 0);
    check(c, hipGetLastError());
  }
  record(c, 4);

  // ---------------------------------------------------------------- a4 --
  int64_t Ptot = 0;
  c.emit_blocks = 0;  // set by the blocked emission when it runs
  double stream_ms = 0;                 // streamed emission (count-only calls)
  std::vector<int64_t> stream_n;        // per pair: pairs streamed
  std::vector<uint64_t> stream_chk;     // per pair: checksum of the streamed records
  bool timed = false, emitted = false;
  int fused = 0;  // work list: 0 round by round, 1 in one workgroup, -1 out of room there
  int32_t* derr = need<int32_t>(c, c.err, 64);
  fill_u32((uint32_t*)derr, 0, 1, st);
  if (N >= 2) {
    const WspdTuning& tun = c.tun;
    uint32_t* rflag = need<uint32_t>(c, c.head, N - 1);
    launch_wspd_roots_flags(T, rflag, st);
    uint32_t* rpos = scan_flags(c, rflag, N - 1, c.idx);
    int64_t f = (int64_t)total_of(c, rflag, rpos, N - 1);
    int2* F = need<int2>(c, c.itemsA, f);
    launch_wspd_roots_fill(T, rflag, rpos, F, st);
    if (f > 1) {  // canonical root order: (rep left, rep right)
      uint64_t* rkeys = need<uint64_t>(c, c.kw0, f);
      launch_item_keys(T, F, f, true, rkeys, st);
      uint32_t* rperm;
      uint64_t* rtop;
      const uint64_t* rw[1] = {rkeys};
      sort_words(c, rw, 1, f, &rperm, &rtop);
      int2* F2 = need<int2>(c, c.itemsB, f);
      launch_gather_items(F, rperm, F2, f, st);
      std::swap(c.itemsA, c.itemsB);
      F = (int2*)c.itemsA.p;
    }
    int64_t isz = 0;
    int2* I = need<int2>(c, c.itemsI, std::max<int64_t>(f, 1024));
    check(c, hipEventRecord(c.kev[0], st));
    trace(c, "root items", f);
    constexpr int kMaxRounds = 4 * 64 + 8;  // deeper than two 64-bit key trees
    if (f > 0 && N <= c.fused_expand_cells) {
      fused = -1;
      // a small launch group: every round in one workgroup, one wait; if its
      // buffers run out, the rounds below run one by one from the roots
      const int64_t capk = c.fused_expand_items > 0 ? c.fused_expand_items : 64 * N + 4096;
      const int64_t capf = c.fused_expand_items > 0 ? c.fused_expand_items : 16 * N + 4096;
      int2* kept = need<int2>(c, c.itemsI, capk);
      int2* fa = need<int2>(c, c.itemsB, capf);
      int2* fb = need<int2>(c, c.itemsX, capf);
      int64_t* ctl = (int64_t*)need<uint64_t>(c, c.small, 64) + 16;
      launch_wspd_expand_small(T, F, f, s, tun, (const int32_t*)c.pcap.p, prune, l2, kMaxRounds, kept, capk, fa, fb,
                               capf, ctl, st);
      check(c, hipGetLastError());
      readback(c, ctl, (int64_t*)c.hpin, 2);
      const int64_t got = (int64_t)c.hpin[0], status = (int64_t)c.hpin[1];
      if (status == 2) throw StageError{W1_EOVERFLOW};
      trace(c, "fused expansion (0 done, 1 out of room)", status);
      I = kept;  // the same buffer the rounds below fill on a fallback
      if (status == 0) {
        fused = 1;
        isz = got;
        f = 0;
        trace(c, "  kept items", isz);
      }
    }
    for (int round = 0; f > 0; ++round) {
      if (round > kMaxRounds) throw StageError{W1_EOVERFLOW};
      if (!worklist_round_fits(f)) throw StageError{W1_EOVERFLOW};
      uint64_t* cnt = need<uint64_t>(c, c.icnt, f);
      uint64_t* pos = need<uint64_t>(c, c.ipos, f);
      launch_wspd_classify(T, F, f, s, tun, (const int32_t*)c.pcap.p, prune, l2, cnt, st);
      scan_u64(cnt, pos, f, need<char>(c, c.scantmp, (int64_t)scan_tmp_bytes(f, 8)), st);
      uint64_t* slot = need<uint64_t>(c, c.small, 64);
      launch_count_total64(cnt, pos, f, slot, st);
      const uint64_t tot = read_u64(c, slot);
      const int64_t kept = (int64_t)(uint32_t)tot, grown = (int64_t)(tot >> 32);
      if (!worklist_items_fit(isz + kept)) throw StageError{W1_EOVERFLOW};
      I = grow_keep<int2>(c, c.itemsI, isz + kept, isz);
      int2* Nx = need<int2>(c, c.itemsB, std::max<int64_t>(grown, 1));
      F = (int2*)c.itemsA.p;
      launch_wspd_scatter(T, F, f, cnt, pos, I, isz, l2, Nx, st);
      check(c, hipGetLastError());
      std::swap(c.itemsA, c.itemsB);
      F = (int2*)c.itemsA.p;
      isz += kept;
      f = grown;
      trace(c, "  round: kept items", isz);
      trace(c, "  round: frontier", f);
    }
    const int64_t m = isz;
    if (m > 0) {
      // A short work list is cut into shorter chunks, so that every wave of
      // the passes gets some: a chunk is walked by one wave, and with fewer
      // chunks than waves the passes last as long as the longest chunk (on a
      // 400 + 400-point pair ~0.5 ms each for ~40 chunks of 512 items).  The
      // pairs are the same for any chunk size; only the order of the records
      // changes, which the sorted network rows and the order-free checksums
      // do not see.
      WspdTuning tg = tun;
      {
        const int64_t waves = (int64_t)c.num_cus * tun.blocks_per_cu * 4;
        while (tg.chunk_items > 16 && m / tg.chunk_items < 2 * waves) tg.chunk_items /= 2;
      }
      // sort items by (rep U, rep V): Morton order, pair-major, canonical
      uint64_t* keys = need<uint64_t>(c, c.kw0, m);
      launch_item_keys(T, I, m, false, keys, st);
      uint32_t* perm;
      uint64_t* top;
      const uint64_t* words[1] = {keys};
      sort_words(c, words, 1, m, &perm, &top);
      int32_t* ipp = need<int32_t>(c, c.ipp, K);
      fill_u64((uint64_t*)P.seg_lo, 0, K, st);
      fill_u64((uint64_t*)P.seg_hi, 0, K, st);
      launch_item_bounds(T.cpair, top, m, P.seg_lo, P.seg_hi, st);
      launch_bounds_count32(P.seg_lo, P.seg_hi, K, ipp, st);
      int2* S = need<int2>(c, c.itemsS, m);  // work entries in sorted order
      launch_item_prep(T, I, perm, m, s, (const int32_t*)c.rmap.p, l2, S, st);
      timed = true;
      std::vector<int32_t> hipp = fetch_pairs(c, ipp, K);
      std::vector<int64_t> ist((size_t)K);
      std::vector<int32_t> cst((size_t)K + 1);
      int64_t acc = 0, nch = 0;
      for (int64_t p = 0; p < K; ++p) {
        ist[(size_t)p] = acc;
        cst[(size_t)p] = (int32_t)nch;
        acc += hipp[(size_t)p];
        nch += (hipp[(size_t)p] + tg.chunk_items - 1) / tg.chunk_items;
      }
      cst[(size_t)K] = (int32_t)nch;
      if (!worklist_chunks_fit(nch)) throw StageError{W1_EOVERFLOW};
      int32_t* cstd = need<int32_t>(c, c.cid, K + 1);
      int32_t hr[9];
      for (int x = 0; x <= 8; ++x) hr[x] = (int32_t)((nch * x) / 8);
      int32_t* xr = need<int32_t>(c, c.xrange, 16);
      upload_all(c, {{P.item_start, ist.data(), (size_t)K * 8},
                     {cstd, cst.data(), (size_t)(K + 1) * 4},
                     {xr, hr, sizeof(hr)}});
      trace(c, "chunks", nch);
      int32_t* cf = need<int32_t>(c, c.cfirst, nch);
      int32_t* ce = need<int32_t>(c, c.cend, nch);
      int32_t* cp = need<int32_t>(c, c.cpairs, nch);
      launch_chunks(cstd, K, P.item_start, ipp, nch, tg.chunk_items, cf, ce, cp, st);
      uint32_t* xc = need<uint32_t>(c, c.xctr, 16);
      uint64_t* ccnt = need<uint64_t>(c, c.ccnt, nch);
      uint64_t* coff = need<uint64_t>(c, c.coff, nch);
      // The network path of a single large pair emits without the count
      // pass: a count over every kSampleStride-th chunk sizes an arena of
      // blocks that the waves fill as they go (the rows are sorted later,
      // so where a record lands does not matter).  If the blocks run out,
      // the counted layout below runs instead.
      bool blocked = false;
      uint32_t nblk = 0;
      const uint32_t brecs = (uint32_t)csr_tile_records();
      if (!(o.flags & W1_COUNT_ONLY) && K == 1 && nch >= kBlockedMinChunks && c.blocked_emit) {
        fill_u64(ccnt, 0, nch, st);
        fill_u32(xc, 0, 8, st);
        check(c, hipEventRecord(c.kev[1], st));
        launch_wspd_pass(false, T, split, S, cf, ce, nch, xr, xc, s, tg, ccnt, coff, nullptr, derr, prune, l2,
                         BucketHist{}, StreamOut{}, BlockOut{}, kSampleStride, c.num_cus, st);
        check(c, hipGetLastError());
        check(c, hipEventRecord(c.kev[2], st));
        scan_u64(ccnt, coff, nch, need<char>(c, c.scantmp, (int64_t)scan_tmp_bytes(nch, 8)), st);
        uint64_t* slot = need<uint64_t>(c, c.small, 64);
        launch_count_total64(ccnt, coff, nch, slot, st);
        const double est = (double)read_u64(c, slot) * kSampleStride;
        const int64_t waves = (int64_t)c.num_cus * tun.blocks_per_cu * 4;
        int64_t cap = (int64_t)std::ceil(est * 1.2 / brecs) + waves + 64;
        if (c.emit_block_limit > 0) cap = std::min(cap, c.emit_block_limit);
        trace(c, "blocked emission: estimated pairs", (int64_t)est);
        if (cap < (int64_t(1) << 31) / 2) {
          const CsrGeometry geo = csr_geometry(N, maxnp);
          if (!geo.ok) throw StageError{W1_ERANGE};
          uint32_t* pout = need<uint32_t>(c, c.pu, 2 * cap * (int64_t)brecs);
          uint32_t* bf = need<uint32_t>(c, c.bfill, cap);
          uint32_t* bp = need<uint32_t>(c, c.bpairs, cap);
          uint32_t* ctl = need<uint32_t>(c, c.bctl, 64);
          fill_u32(ctl, 0, 2, st);  // [0] blocks taken, [1] overflow
          fill_u64(P.npairs, 0, K, st);
          uint64_t* bcnt = need<uint64_t>(c, c.bcnt, geo.NB);
          fill_u64(bcnt, 0, geo.NB, st);
          BucketHist bh;
          bh.chunk_pair = cp;
          bh.cell_start = P.cell_start;
          bh.RB = geo.RB;
          bh.NB = (int)geo.NB;
          bh.count = bcnt;
          BlockOut bo;
          bo.base = pout;
          bo.block = brecs;
          bo.max_blocks = (uint32_t)cap;
          bo.nblocks = ctl;
          bo.fill = bf;
          bo.pair = bp;
          bo.pair_count = (unsigned long long*)P.npairs;
          bo.overflow = (int32_t*)(ctl + 1);
          bo.chunk_pair = cp;
          fill_u32(xc, 0, 8, st);
          check(c, hipEventRecord(c.kev[3], st));
          launch_wspd_pass(true, T, nullptr, S, cf, ce, nch, xr, xc, s, tg, ccnt, coff, nullptr, derr, prune, l2,
                           bh, StreamOut{}, bo, 1, c.num_cus, st);
          check(c, hipGetLastError());
          uint32_t hctl[2];
          readback(c, ctl, hctl, 2);
          if (hctl[1] == 0 && hctl[0] <= (uint32_t)cap) {
            blocked = true;
            emitted = true;
            nblk = hctl[0];
            uint64_t np0 = 0;
            readback(c, P.npairs, &np0, 1);
            Ptot = (int64_t)np0;
            trace(c, "wspd pairs", Ptot);
            trace(c, "blocked emission: blocks", (int64_t)nblk);
          }
        }
      }
      c.emit_blocks = blocked ? nblk : 0;
      c.emit_block_recs = brecs;
      // A short work list on the network path skips the count pass: each
      // chunk writes into a slot of chunk_items * (largest work cap) records
      // (an item covers at most its work cap of leaf pairs, so no chunk can
      // fill more), counting as it goes; the records are then moved to
      // their scanned offsets.  Same records as the counted layout.
      const int64_t slot_recs = (int64_t)tg.chunk_items * maxcap;
      const bool slotted = !blocked && !(o.flags & W1_COUNT_ONLY) && slot_recs > 0 &&
                           nch * slot_recs <= kSlottedMaxRecords;
      if (slotted) {
        const CsrGeometry geo = csr_geometry(N, maxnp);
        if (!geo.ok) throw StageError{W1_ERANGE};
        uint64_t* bcnt = need<uint64_t>(c, c.bcnt, geo.NB);
        fill_u64(bcnt, 0, geo.NB, st);
        BucketHist bh;
        bh.chunk_pair = cp;
        bh.cell_start = P.cell_start;
        bh.RB = geo.RB;
        bh.NB = (int)geo.NB;
        bh.count = bcnt;
        uint32_t* sl = need<uint32_t>(c, c.pslot, 3 * nch * slot_recs);
        StreamOut so;
        so.slot = slot_recs;
        fill_u32(xc, 0, 8, st);
        check(c, hipEventRecord(c.kev[1], st));
        check(c, hipEventRecord(c.kev[2], st));  // no count pass
        check(c, hipEventRecord(c.kev[3], st));
        c.rec_words = launch_wspd_pass(true, T, split, S, cf, ce, nch, xr, xc, s, tg, ccnt, coff, sl, derr, prune, l2,
                                       bh, so, BlockOut{}, 1, c.num_cus, st);
        check(c, hipGetLastError());
        scan_u64(ccnt, coff, nch, need<char>(c, c.scantmp, (int64_t)scan_tmp_bytes(nch, 8)), st);
        uint64_t* slot = need<uint64_t>(c, c.small, 64);
        launch_count_total64(ccnt, coff, nch, slot, st);
        Ptot = (int64_t)read_u64(c, slot);
        trace(c, "wspd pairs (slotted emission)", Ptot);
        fill_u64((uint64_t*)P.seg_hi, 0, K, st);
        launch_pair_totals(ccnt, coff, cp, nch, P.pair_start, (uint64_t*)P.seg_hi, P.npairs, K, st);
        if (Ptot > 0) {
          uint32_t* pout = need<uint32_t>(c, c.pu, std::max<int64_t>(c.rec_words * Ptot, 2 * Ptot + 2 * N + K));
          launch_compact_slots(sl, ccnt, coff, nch, slot_recs, c.rec_words, pout, st);
          check(c, hipGetLastError());
          emitted = true;
        }
      }
      if (!blocked && !slotted) {
      fill_u32(xc, 0, 8, st);
      check(c, hipEventRecord(c.kev[1], st));
      launch_wspd_pass(false, T, split, S, cf, ce, nch, xr, xc, s, tg, ccnt, coff, nullptr, derr, prune, l2,
                       BucketHist{}, StreamOut{}, BlockOut{}, 1, c.num_cus, st);
      check(c, hipGetLastError());
      check(c, hipEventRecord(c.kev[2], st));
      scan_u64(ccnt, coff, nch, need<char>(c, c.scantmp, (int64_t)scan_tmp_bytes(nch, 8)), st);
      uint64_t* slot = need<uint64_t>(c, c.small, 64);
      launch_count_total64(ccnt, coff, nch, slot, st);
      Ptot = (int64_t)read_u64(c, slot);
      trace(c, "wspd pairs", Ptot);
      if (c.trace && nch > 0) {  // the spread of the pairs over the chunks
        std::vector<uint64_t> hc((size_t)nch);
        readback(c, ccnt, hc.data(), nch);
        std::vector<uint64_t> sorted_c(hc);
        std::sort(sorted_c.begin(), sorted_c.end());
        trace(c, "  pairs per chunk: max", (int64_t)sorted_c.back());
        trace(c, "  pairs per chunk: 99.9th percentile", (int64_t)sorted_c[(size_t)((nch - 1) * 999 / 1000)]);
        trace(c, "  pairs per chunk: median", (int64_t)sorted_c[(size_t)(nch / 2)]);
        uint64_t smax = 0;
        for (int64_t k = 0; k < nch; k += kSampleStride) smax = std::max(smax, hc[(size_t)k]);
        trace(c, "  pairs per chunk: max over every 16th chunk", (int64_t)smax);
      }
      fill_u64((uint64_t*)P.seg_hi, 0, K, st);
      launch_pair_totals(ccnt, coff, cp, nch, P.pair_start, (uint64_t*)P.seg_hi, P.npairs, K, st);
      if ((o.flags & W1_COUNT_ONLY) && c.stream_arena > 0 && Ptot > 0) {
        // streamed emission: runs of consecutive chunks whose pairs fit the
        // arena, each run written over the previous one, with per-chunk
        // checksums of the records
        std::vector<uint64_t> hoff((size_t)nch), hcnt((size_t)nch);
        readback(c, coff, hoff.data(), nch);
        readback(c, ccnt, hcnt.data(), nch);
        uint32_t* arena = need<uint32_t>(c, c.pu, 3 * c.stream_arena);
        uint64_t* csum = need<uint64_t>(c, c.csum, 2 * nch);
        fill_u64(csum, 0, 2 * nch, st);
        // the arena fills, planned on the host: chunk ranges per XCD and the
        // first pair of each run
        std::vector<int32_t> run_xr;
        std::vector<int64_t> run_base;
        int64_t c0 = 0;
        for (int round = 0; c0 < nch && (c.stream_rounds == 0 || round < c.stream_rounds); ++round) {
          int64_t c1 = c0;
          while (c1 < nch && hoff[(size_t)c1] + hcnt[(size_t)c1] - hoff[(size_t)c0] <= (uint64_t)c.stream_arena) ++c1;
          if (c1 == c0) throw StageError{W1_EOVERFLOW};  // one chunk holds more pairs than the arena
          for (int x = 0; x <= 8; ++x) run_xr.push_back((int32_t)(c0 + ((c1 - c0) * x) / 8));
          run_base.push_back((int64_t)hoff[(size_t)c0]);
          c0 = c1;
        }
        const int nruns = (int)run_base.size();
        int32_t* dxr = need<int32_t>(c, c.runxr, 9 * (int64_t)nruns);
        int64_t* dtab = need<int64_t>(c, c.runbase, (int64_t)nruns + 2);  // bases, current base, fill counter
        upload_all(c, {{dxr, run_xr.data(), run_xr.size() * 4}, {dtab, run_base.data(), run_base.size() * 8}});
        int64_t* cur_base = dtab + nruns;
        int32_t* ctr = (int32_t*)(dtab + nruns + 1);
        fill_u32((uint32_t*)ctr, 0, 1, st);
        const StreamOut so{0, cur_base, csum};
        // one arena fill: the next run's ranges and base, then the emit pass
        auto fill_once = [&](hipStream_t s2) {
          launch_stream_next(dxr, dtab, nruns, ctr, xr, cur_base, xc, s2);
          launch_wspd_pass(true, T, nullptr, S, cf, ce, nch, xr, xc, s, tg, ccnt, coff, arena, derr, prune, l2,
                           BucketHist{}, so, BlockOut{}, 1, c.num_cus, s2);
        };
        GraphGuard gg;
        if (c.stream_graph && nruns > 1) {
          // captured once on a private stream, replayed on the caller's for
          // every fill: no host wait between fills (the graph holds kernels
          // only, no memset nodes)
          check(c, hipStreamCreateWithFlags(&gg.cap, hipStreamNonBlocking));
          gg.wait = st;
          check(c, hipStreamBeginCapture(gg.cap, hipStreamCaptureModeThreadLocal));
          gg.capturing = true;
          fill_once(gg.cap);
          gg.capturing = false;
          check(c, hipStreamEndCapture(gg.cap, &gg.graph));
          check(c, hipGraphInstantiate(&gg.exec, gg.graph, nullptr, nullptr, 0));
        }
        check(c, hipEventRecord(c.kev[3], st));
        for (int r = 0; r < nruns; ++r) {
          if (gg.exec) check(c, hipGraphLaunch(gg.exec, st));
          else fill_once(st);
        }
        check(c, hipGetLastError());
        check(c, hipEventRecord(c.kev[4], st));
        check(c, hipEventSynchronize(c.kev[4]));
        float ms = 0;
        (void)hipEventElapsedTime(&ms, c.kev[3], c.kev[4]);
        stream_ms = ms;
        std::vector<uint64_t> hsum((size_t)(2 * c0));
        std::vector<int32_t> hcp((size_t)c0);
        readback(c, csum, hsum.data(), 2 * c0);
        readback(c, cp, hcp.data(), c0);
        stream_n.assign((size_t)K, 0);
        stream_chk.assign((size_t)(2 * K), 0);
        for (int64_t k = 0; k < c0; ++k) {
          const size_t p = (size_t)hcp[(size_t)k];
          stream_n[p] += (int64_t)hcnt[(size_t)k];
          stream_chk[2 * p] += hsum[(size_t)(2 * k)];
          stream_chk[2 * p + 1] += hsum[(size_t)(2 * k + 1)];
        }
      }
      if (!(o.flags & W1_COUNT_ONLY) && Ptot > 0) {
        // the records' buffer later holds the rows' unsorted heads, which
        // are placed by final arc number (2 Ptot WSPD arcs plus at most
        // 2 N + K diagonal arcs); records are (u, v) when the packed split
        // records exist, else (u, v, cost)
        uint32_t* pout = need<uint32_t>(c, c.pu, std::max<int64_t>((split ? 2 : 3) * Ptot, 2 * Ptot + 2 * N + K));
        // the emit pass also counts the arcs per tail bucket of the
        // network's row partition (a5)
        const CsrGeometry geo = csr_geometry(N, maxnp);
        if (!geo.ok) throw StageError{W1_ERANGE};
        uint64_t* bcnt = need<uint64_t>(c, c.bcnt, geo.NB);
        fill_u64(bcnt, 0, geo.NB, st);
        BucketHist bh;
        bh.chunk_pair = cp;
        bh.cell_start = P.cell_start;
        bh.RB = geo.RB;
        bh.NB = (int)geo.NB;
        bh.count = bcnt;
        fill_u32(xc, 0, 8, st);
        check(c, hipEventRecord(c.kev[3], st));
        c.rec_words = launch_wspd_pass(true, T, split, S, cf, ce, nch, xr, xc, s, tg, ccnt, coff, pout, derr, prune,
                                       l2, bh, StreamOut{}, BlockOut{}, 1, c.num_cus, st);
        check(c, hipGetLastError());
        emitted = true;
      }
      }  // counted layout
    }
  }
  record(c, 5);
  for (double& x : c.kms) x = 0;
  c.kms[3] = (double)Ptot;
  c.kms[4] = stream_ms;
  c.kms[9] = (double)c.emit_blocks;
  c.kms[10] = (double)fused;
  c.kms[11] = emitted ? (double)(c.emit_blocks > 0 ? 2 : c.rec_words) : 0.0;

  // ---------------------------------------------------------------- a5 --
  // The network in compressed sparse row form, sorted by (tail, head)
  // (Appendix, network representation); see csr.hip for the passes.
  bool csr_timed = false;
  int64_t Mtot = 0;
  std::vector<int32_t> h_costK;  // Euclidean cost scale per pair
  std::vector<uint64_t> h_parc;  // first arc of each pair, then the total
  if (N > 0 && !(o.flags & W1_COUNT_ONLY)) {
    const uint32_t* cp = (const uint32_t*)c.cpair.p;
    const int2* cij = (const int2*)c.cij.p;
    const int32_t* ca = (const int32_t*)c.ca.p;
    const int32_t* cb = (const int32_t*)c.cb.p;
    const int32_t* ncl = P.ncells;
    const CsrGeometry geo = csr_geometry(N, maxnp);
    if (!geo.ok) throw StageError{W1_ERANGE};
    const int RB = geo.RB, DB = geo.DB;
    const int64_t NB = geo.NB;
    trace(c, "csr bucket rows (log2)", RB);
    trace(c, "csr head bits", DB);
    const int64_t NR = N + 2 * K;  // rows: cells plus two diagonal nodes per pair
    uint32_t* heads = (uint32_t*)c.pu.p;
    uint32_t* col = need<uint32_t>(c, c.l1, 2 * Ptot + 2 * N + K);
    uint32_t* rowcnt = need<uint32_t>(c, c.rowcnt, N);
    fill_u32(rowcnt, 0, N, st);
    int64_t* sup = need<int64_t>(c, c.supply, NR);
    int64_t ntiles = 0, ntiles_h = 0;  // tiles of the row scatter and of the row histogram
    const uint64_t* bstart = nullptr;
    const int64_t* tfirst = nullptr;
    if (Ptot > 0) {
      uint64_t* rstart = need<uint64_t>(c, c.rstart, K);
      scan_u64(P.npairs, rstart, K, need<char>(c, c.scantmp, (int64_t)scan_tmp_bytes(K, 8)), st);
      const uint64_t* bcnt = (const uint64_t*)c.bcnt.p;  // taken by the emit pass
      csr_timed = true;
      check(c, hipEventRecord(c.kev[4], st));
      check(c, hipEventRecord(c.kev[5], st));
      // bucket starts and the tiles of the row passes (host: NB is small)
      std::vector<uint64_t> hb((size_t)NB);
      readback(c, bcnt, hb.data(), NB);
      // (the row histogram takes larger tiles than the row scatter: its only
      // per-tile cost is one atomic per row of the bucket)
      const int64_t et = csr_entry_tile(RB), eth = csr_hist_tile(RB);
      std::vector<uint64_t> hbs((size_t)NB + 1);
      std::vector<int64_t> htf((size_t)(2 * (NB + 1)));
      uint64_t acc = 0;
      for (int64_t b = 0; b < NB; ++b) {
        hbs[(size_t)b] = acc;
        htf[(size_t)b] = ntiles;
        htf[(size_t)(NB + 1 + b)] = ntiles_h;
        acc += hb[(size_t)b];
        ntiles += ceil_div((int64_t)hb[(size_t)b], et);
        ntiles_h += ceil_div((int64_t)hb[(size_t)b], eth);
      }
      hbs[(size_t)NB] = acc;
      htf[(size_t)NB] = ntiles;
      htf[(size_t)(2 * NB + 1)] = ntiles_h;
      if (acc != 2 * (uint64_t)Ptot || ntiles >= (int64_t(1) << 31)) throw StageError{W1_EOVERFLOW};
      uint64_t* dbs = need<uint64_t>(c, c.bstart, NB + 1);
      int64_t* dtf = need<int64_t>(c, c.tfirst, 2 * (NB + 1));
      upload_all(c, {{dbs, hbs.data(), (size_t)(NB + 1) * 8}, {dtf, htf.data(), (size_t)(2 * (NB + 1)) * 8}});
      bstart = dbs;
      tfirst = dtf;
      uint64_t* bcur = need<uint64_t>(c, c.bcur, NB * csr_bucket_stride());
      fill_u64(bcur, 0, NB * csr_bucket_stride(), st);
      check(c, hipEventRecord(c.kev[6], st));
      const bool blk = c.emit_blocks > 0;
      launch_csr_bucket_scatter((const uint32_t*)c.pu.p, c.rec_words, (uint64_t)Ptot, rstart, K, P.cell_start, RB, DB,
                                (int)NB, bstart, bcur, col, blk ? (const uint32_t*)c.bfill.p : nullptr,
                                blk ? (const uint32_t*)c.bpairs.p : nullptr, c.emit_block_recs, c.emit_blocks, st);
      check(c, hipEventRecord(c.kev[7], st));
      launch_csr_row_hist(col, tfirst + NB + 1, ntiles_h, (int)NB, bstart, RB, DB, N, rowcnt, st);
      check(c, hipEventRecord(c.kev[8], st));
    }
    // degrees, row offsets
    uint32_t* bflag = need<uint32_t>(c, c.bflag, N);
    launch_csr_bflags(cb, N, bflag, st);
    uint32_t* bpos = scan_flags(c, bflag, N, c.bpos);
    uint64_t* deg = need<uint64_t>(c, c.deg, NR + 1);
    fill_u64(deg, 0, NR + 1, st);
    launch_csr_row_deg(cp, P.cell_start, ncl, ca, cb, rowcnt, bpos, N, deg, st);
    uint64_t* off = need<uint64_t>(c, c.off, NR + 1);
    scan_u64(deg, off, NR + 1, need<char>(c, c.scantmp, (int64_t)scan_tmp_bytes(NR + 1, 8)), st);
    if (Ptot > 0) {
      uint32_t* rowcur = need<uint32_t>(c, c.rowcur, N);
      fill_u32(rowcur, 0, N, st);
      // the pair records are consumed: their buffer takes the rows' heads
      heads = need<uint32_t>(c, c.pu, 2 * Ptot + 2 * N + K);
      launch_csr_row_scatter(col, tfirst, ntiles, (int)NB, bstart, RB, DB, N, cp, off, rowcur, heads, st);
      check(c, hipEventRecord(c.kev[9], st));
    }
    // Euclidean costs: 64-bit, in units of g 2^-K with K per pair from the
    // pair's point count n and largest shifted coordinate X:
    // K = min(30, 59 - bitlen(n) - bitlen(X)), so F* and the flow solver's
    // artificial costs stay below 2^60
    const int32_t* costK = nullptr;
    if (l2) {
      uint64_t* xm = need<uint64_t>(c, c.pxmax, K);
      fill_u64(xm, 0, K, st);
      launch_pair_xmax(cp, cij, N, xm, st);
      std::vector<uint64_t> hx((size_t)K);
      std::vector<int64_t> hna((size_t)K), hnb((size_t)K);
      check(c, hipMemcpyAsync(hna.data(), P.nA, (size_t)K * 8, hipMemcpyDeviceToHost, st));
      check(c, hipMemcpyAsync(hnb.data(), P.nB, (size_t)K * 8, hipMemcpyDeviceToHost, st));
      readback(c, xm, hx.data(), K);
      std::vector<int32_t> hk((size_t)K);
      for (int64_t p = 0; p < K; ++p) {
        const int64_t k = std::min<int64_t>(
            30, 59 - bitlen_u64((uint64_t)(hna[(size_t)p] + hnb[(size_t)p])) - bitlen_u64(std::max<uint64_t>(hx[(size_t)p], 1)));
        if (k < 0) throw StageError{W1_ERANGE};
        hk[(size_t)p] = (int32_t)k;
      }
      upload(c, P.costK, hk.data(), (size_t)K * 4);
      costK = P.costK;
      h_costK = hk;
    }
    void* cost = l2 ? (void*)need<int64_t>(c, c.costb, 2 * Ptot + 2 * N + K)
                    : (void*)need<int32_t>(c, c.costb, 2 * Ptot + 2 * N + K);
    uint64_t* rowq = need<uint64_t>(c, c.rowq, 1);
    fill_u64(rowq, 0, 1, st);
    launch_csr_row_sort(cp, P.cell_start, ncl, cij, ca, rowcnt, off, heads, N, maxnp, c.sort_window, c.num_cus, costK,
                        col, cost, rowq, st);
    launch_csr_bdiag(cp, P.cell_start, ncl, cij, ca, cb, bpos, off, P, N, costK, col, cost, sup, st);
    int64_t* rp = need<int64_t>(c, c.rp, N + 3 * K);
    fill_u64((uint64_t*)rp, 0, N + 3 * K, st);
    launch_csr_local_rowptr(cp, P.cell_start, ncl, off, N, rp, st);
    uint64_t* parc = need<uint64_t>(c, c.parc, K + 1);
    launch_csr_pair_arcs(P.cell_start, off, K, NR, parc, st);
    check(c, hipEventRecord(c.kev[10], st));
    check(c, hipGetLastError());
    h_parc.resize((size_t)K + 1);  // read with the per-pair arrays below
    check(c, hipMemcpyAsync(h_parc.data(), parc, (size_t)(K + 1) * 8, hipMemcpyDeviceToHost, st));
  }
  record(c, 6);
  // the arcs per pair, the traversal's overflow flag and every per-pair
  // array: one wait
  std::vector<char> hpb((size_t)c.pair_bytes);
  check(c, hipMemcpyAsync(c.hpin, derr, 4, hipMemcpyDeviceToHost, st));
  readback(c, (const char*)c.pairs.p, hpb.data(), c.pair_bytes);
  int32_t herr = 0;
  std::memcpy(&herr, c.hpin, 4);
  if (!h_parc.empty()) {
    Mtot = (int64_t)h_parc[(size_t)K];
    trace(c, "network arcs", Mtot);
  }
  if (timed) {
    float a = 0, b2 = 0, d = 0;
    (void)hipEventElapsedTime(&a, c.kev[0], c.kev[1]);
    (void)hipEventElapsedTime(&b2, c.kev[1], c.kev[2]);
    if (emitted) (void)hipEventElapsedTime(&d, c.kev[3], c.ev[5]);
    c.kms[0] = a;
    c.kms[1] = b2;
    c.kms[2] = d;
  }
  if (csr_timed) {
    float t[5] = {0, 0, 0, 0, 0};
    (void)hipEventElapsedTime(&t[0], c.kev[4], c.kev[5]);
    (void)hipEventElapsedTime(&t[1], c.kev[6], c.kev[7]);
    (void)hipEventElapsedTime(&t[2], c.kev[7], c.kev[8]);
    (void)hipEventElapsedTime(&t[3], c.kev[8], c.kev[9]);
    (void)hipEventElapsedTime(&t[4], c.kev[9], c.kev[10]);
    for (int i = 1; i < 5; ++i) c.kms[4 + i] = t[i];
  }
  if (herr) throw StageError{W1_EOVERFLOW};

  // ------------------------------------------------------------ results --
  auto host = [&](const auto* dev) { return from_pair_block(c, hpb, dev, K); };
  std::vector<int32_t> h_err = host(P.err), h_locA = host(P.locA), h_locB = host(P.locB), h_e = host(P.e),
                       h_nc = host(P.ncells), h_FA = host(P.FA), h_FB = host(P.FB);
  std::vector<int64_t> h_nA = host(P.nA), h_nB = host(P.nB), h_cs = host(P.cell_start);
  std::vector<uint64_t> h_sA = host(P.sumA), h_sB = host(P.sumB), h_np = host(P.npairs);
  std::vector<double> h_L = host(P.L);
  float tms[8] = {0};
  for (int i = 0; i < 6; ++i) (void)hipEventElapsedTime(&tms[i], c.ev[i], c.ev[i + 1]);
  c.h_cell_start.assign(h_cs.begin(), h_cs.end());
  c.h_ncells.assign(h_nc.begin(), h_nc.end());
  c.h_npairs.assign(h_np.begin(), h_np.end());
  c.h_arc_start.assign((size_t)K, 0);
  c.h_narcs.assign((size_t)K, 0);
  if (!h_parc.empty())
    for (int64_t p = 0; p < K; ++p) {
      c.h_arc_start[(size_t)p] = (int64_t)h_parc[(size_t)p];
      c.h_narcs[(size_t)p] = (int64_t)(h_parc[(size_t)p + 1] - h_parc[(size_t)p]);
    }
  c.network_valid = !(o.flags & W1_COUNT_ONLY);
  c.network_l2 = l2;
  int64_t loc_off = 0;
  for (int64_t p = 0; p < K; ++p) {
    w1_result& r = res[p];
    std::memset(&r, 0, sizeof(r));
    r.s = s;
    r.status = h_err[(size_t)p];
    r.flow_cost = -1;
    r.n_a = h_nA[(size_t)p];
    r.n_b = h_nB[(size_t)p];
    r.n_points = r.n_a + r.n_b;
    r.n_locations = (int64_t)h_locA[(size_t)p] + h_locB[(size_t)p];
    r.lower_bound = h_L[(size_t)p];
    r.grid_exp = h_e[(size_t)p];
    r.grid = std::ldexp(1.0, r.grid_exp);
    r.n_cells = h_nc[(size_t)p];
    r.n_pairs = (int64_t)h_np[(size_t)p];
    r.n_arcs = c.h_narcs[(size_t)p];
    r.n_diag = r.n_arcs > 0 ? r.n_arcs - 2 * r.n_pairs : 0;
    r.rwmd_sum_a = (int64_t)h_sA[(size_t)p];
    r.rwmd_sum_b = (int64_t)h_sB[(size_t)p];
    r.rwmd_shift_a = h_FA[(size_t)p];
    r.rwmd_shift_b = h_FB[(size_t)p];
    r.metric_l2 = l2 ? 1 : 0;
    r.cost_shift = h_costK.empty() ? 0 : h_costK[(size_t)p];
    if (!stream_n.empty()) {
      r.n_pairs_streamed = stream_n[(size_t)p];
      r.pair_checksum[0] = stream_chk[2 * (size_t)p];
      r.pair_checksum[1] = stream_chk[2 * (size_t)p + 1];
    }
    for (int i = 0; i < 6; ++i) r.t_ms[i] = tms[i];
    if (r.status == 0 && r.n_points == 0) {
      r.w1 = r.w1_paper = 0.0;
      r.flow_cost = 0;
      r.flow_solved = 1;
    }
    // stage intermediates
    if ((o.flags & W1_KEEP_STAGES) && r.status == 0 && r.n_locations > 0) {
      const int64_t nl = r.n_locations;
      r.loc_b = (double*)std::malloc((size_t)nl * 8);
      r.loc_d = (double*)std::malloc((size_t)nl * 8);
      r.loc_t = (double*)std::malloc((size_t)nl * 8);
      r.loc_w = (int32_t*)std::malloc((size_t)nl * 4);
      if (!r.loc_b || !r.loc_d || !r.loc_t || !r.loc_w) throw StageError{W1_ENOMEM};
      readback(c, (const double*)c.lb.p + loc_off, r.loc_b, nl);
      readback(c, (const double*)c.ld.p + loc_off, r.loc_d, nl);
      readback(c, (const double*)c.lt.p + loc_off, r.loc_t, nl);
      readback(c, (const int32_t*)c.lw.p + loc_off, r.loc_w, nl);
      if (K == 1 && N >= 2) {
        const int64_t ni = N - 1;
        std::vector<int4> aux((size_t)ni), box((size_t)ni);
        readback(c, (const int4*)c.iaux.p, aux.data(), ni);
        readback(c, (const int4*)c.ibox.p, box.data(), ni);
        r.node_lo = (int32_t*)std::malloc((size_t)ni * 4);
        r.node_hi = (int32_t*)std::malloc((size_t)ni * 4);
        r.node_left = (int32_t*)std::malloc((size_t)ni * 4);
        r.node_right = (int32_t*)std::malloc((size_t)ni * 4);
        r.node_box = (int32_t*)std::malloc((size_t)ni * 16);
        if (!r.node_lo || !r.node_hi || !r.node_left || !r.node_right || !r.node_box) throw StageError{W1_ENOMEM};
        for (int64_t q = 0; q < ni; ++q) {
          r.node_left[q] = aux[(size_t)q].x;
          r.node_right[q] = aux[(size_t)q].y;
          r.node_lo[q] = aux[(size_t)q].z;
          r.node_hi[q] = aux[(size_t)q].w;
          std::memcpy(r.node_box + 4 * q, &box[(size_t)q], 16);
        }
      }
    }
    loc_off += (int64_t)h_locA[(size_t)p] + h_locB[(size_t)p];
  }
  (void)Mtot;
  return W1_OK;
}

// Copy one pair's network to the host (arrays owned by the result): cells,
// supplies and the sorted rows (row pointers local to the pair, local node
// ids as heads).
void copy_network(Ctx& c, int64_t p, w1_result& r, std::vector<int2>& ij) {
  const int64_t nc = c.h_ncells[(size_t)p], m = c.h_narcs[(size_t)p];
  const int64_t cs = c.h_cell_start[(size_t)p], as = c.h_arc_start[(size_t)p];
  r.cell_i = (int32_t*)std::malloc((size_t)std::max<int64_t>(nc, 1) * 4);
  r.cell_j = (int32_t*)std::malloc((size_t)std::max<int64_t>(nc, 1) * 4);
  r.cell_ca = (int32_t*)std::malloc((size_t)std::max<int64_t>(nc, 1) * 4);
  r.cell_cb = (int32_t*)std::malloc((size_t)std::max<int64_t>(nc, 1) * 4);
  r.supply = (int64_t*)std::malloc((size_t)(nc + 2) * 8);
  r.row_ptr = (int64_t*)std::malloc((size_t)(nc + 3) * 8);
  r.col = (uint32_t*)std::malloc((size_t)std::max<int64_t>(m, 1) * 4);
  if (r.metric_l2) r.cost64 = (int64_t*)std::malloc((size_t)std::max<int64_t>(m, 1) * 8);
  else r.cost = (int32_t*)std::malloc((size_t)std::max<int64_t>(m, 1) * 4);
  if (!r.cell_i || !r.cell_j || !r.cell_ca || !r.cell_cb || !r.supply || !r.row_ptr || !r.col || !(r.cost || r.cost64))
    throw StageError{W1_ENOMEM};
  // the copies are only queued here: the caller waits once for every pair
  // of the launch group, then finish_network() splits the cell coordinates
  auto get = [&](void* host, const void* dev, size_t bytes) {
    if (bytes) check(c, hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, c.st));
  };
  ij.assign((size_t)std::max<int64_t>(nc, 0), int2{0, 0});
  if (nc > 0) {
    get(ij.data(), (const int2*)c.cij.p + cs, (size_t)nc * 8);
    get(r.cell_ca, (const int32_t*)c.ca.p + cs, (size_t)nc * 4);
    get(r.cell_cb, (const int32_t*)c.cb.p + cs, (size_t)nc * 4);
    get(r.supply, (const int64_t*)c.supply.p + cs + 2 * p, (size_t)(nc + 2) * 8);
    get(r.row_ptr, (const int64_t*)c.rp.p + cs + 3 * p, (size_t)(nc + 3) * 8);
  } else {
    r.supply[0] = r.supply[1] = 0;
    r.row_ptr[0] = r.row_ptr[1] = r.row_ptr[2] = 0;
  }
  if (m > 0) {
    get(r.col, (const uint32_t*)c.l1.p + as, (size_t)m * 4);
    if (r.metric_l2) get(r.cost64, (const int64_t*)c.costb.p + as, (size_t)m * 8);
    else get(r.cost, (const int32_t*)c.costb.p + as, (size_t)m * 4);
  }
}

void finish_network(w1_result& r, const std::vector<int2>& ij) {
  for (int64_t q = 0; q < r.n_cells; ++q) {
    r.cell_i[q] = ij[(size_t)q].x;
    r.cell_j[q] = ij[(size_t)q].y;
  }
}

void free_network(w1_result& r) {
  void* ptrs[] = {r.cell_i, r.cell_j, r.cell_ca, r.cell_cb, r.supply, r.row_ptr, r.col, r.cost, r.cost64};
  for (void* q : ptrs) std::free(q);
  r.cell_i = r.cell_j = r.cell_ca = r.cell_cb = nullptr;
  r.supply = nullptr;
  r.row_ptr = nullptr;
  r.col = nullptr;
  r.cost = nullptr;
  r.cost64 = nullptr;
}

// Flow outcome into the result.  An optimal flow gives the certified w1.  A
// stalled solve (pivot cap) whose flow meets every supply still gives an
// upper bound (any feasible flow costs at least the optimum), but not the
// (1 + eps) guarantee; one that left supply on artificial arcs gives no
// value at all (w1 = w1_paper = NaN, flow_cost = -1, flow_solved = 0).
void finish_flow(w1_result& r, const FlowResult& fr) {
  r.pivots = fr.pivots;
  r.status = fr.status ? W1_STALLED : W1_OPTIMAL;
  if (!fr.feasible) {
    r.flow_cost = -1;
    r.flow_solved = 0;
    r.w1 = r.w1_paper = NAN;
    return;
  }
  r.flow_cost = fr.cost;
  r.flow_solved = 1;
  if (r.metric_l2) {  // g (F* 2^-K + n R): the condensation's n g / sqrt(2) added back
    r.w1_paper = std::ldexp((double)fr.cost, r.grid_exp - r.cost_shift);
    r.w1 = r.w1_paper + (double)r.n_points * std::ldexp(0x1.6a09e667f3bcdp-1, r.grid_exp);
  } else {
    r.w1 = std::ldexp((double)(fr.cost + r.n_points), r.grid_exp - 1);
    r.w1_paper = std::ldexp((double)fr.cost, r.grid_exp - 1);
  }
}

// The host flow leaves out the dominated cell arcs (drop_dominated_arcs in
// flow.cpp states when and why that keeps the optimum).
// Host flow of one pair from its host network copy (the sorted rows are
// the solver's own input form), without the dominated cell arcs.
void solve_flow(w1_result& r, int64_t pivot_cap) {
  FlowResult fr{};
  // the rows are sorted by head and the diagonal nodes come last: the solve
  // starts from the flow through the diagonal
  int rc;
  if (r.metric_l2) {
    SolveRows<int64_t> sr;
    drop_dominated_arcs(r.n_cells, r.row_ptr, r.col, r.cost64, r.cell_i, r.cell_j, r.cost_shift, sr);
    rc = network_simplex64_diag(r.n_cells + 2, sr.row_ptr.data(), sr.col.data(), sr.cost.data(), r.supply, pivot_cap,
                                &fr);
  } else {
    SolveRows<int32_t> sr;
    drop_dominated_arcs(r.n_cells, r.row_ptr, r.col, r.cost, r.cell_i, r.cell_j, -1, sr);
    rc = network_simplex_diag(r.n_cells + 2, sr.row_ptr.data(), sr.col.data(), sr.cost.data(), r.supply, pivot_cap,
                              &fr);
  }
  if (rc != 0) {
    r.status = rc == -3 ? W1_ENOMEM : W1_EINVAL;
    return;
  }
  finish_flow(r, fr);
}

int entry(Ctx* c, const w1_pd* a, const w1_pd* b, int64_t K, const w1_params* params, void* stream, w1_result* out,
          double* L_only) {
  if (!c || !a || !b || K <= 0 || (!out && !L_only)) return W1_EINVAL;
  Opts o;
  if (params) {
    o.eps = params->eps;
    o.kappa = params->cond_frac > 0 ? params->cond_frac : 0.1;
    o.s = params->s_override;
    o.flags = params->flags;
    o.pivot_cap = params->pivot_cap;
    if (params->s_override < 0) return W1_EINVAL;
  }
  if (!(o.eps > 0.0 && o.eps <= 1.0) || !(o.kappa > 0.0 && o.kappa < 0.5)) return W1_EINVAL;
  if (hipSetDevice(c->device) != hipSuccess) return W1_EHIP;
  if (out) std::memset(out, 0, sizeof(w1_result) * (size_t)K);
  try {
    // Launch groups: consecutive pairs whose points fit the per-launch
    // budget (a single pair may exceed it).  Every stage runs once per group.
    for (int64_t g0 = 0; g0 < K;) {
      int64_t g1 = g0, pts = 0;
      while (g1 < K && (g1 == g0 || pts + a[g1].n + b[g1].n <= c->max_points)) {
        pts += a[g1].n + b[g1].n;
        ++g1;
      }
      const int64_t Kg = g1 - g0;
      w1_result* og = out ? out + g0 : nullptr;
      c->K_base = g0;
      int rc = run(*c, a + g0, b + g0, Kg, o, (hipStream_t)stream, og, L_only ? L_only + g0 : nullptr);
      if (rc != W1_OK) {
        if (out)
          for (int64_t p = g1; p < K; ++p) out[p].status = rc;
        return rc;
      }
      g0 = g1;
      if (L_only) continue;
      const bool want_flow = !(o.flags & (W1_COUNT_ONLY | W1_NO_FLOW));
      const bool keep = (o.flags & W1_KEEP_NETWORK) != 0;
      if (!(want_flow || keep)) continue;
      auto t0 = std::chrono::steady_clock::now();
      std::vector<std::vector<int2>> ijs((size_t)Kg);
      for (int64_t p = 0; p < Kg; ++p)
        if (og[p].status == 0 && og[p].n_points > 0) copy_network(*c, p, og[p], ijs[(size_t)p]);
      check(*c, hipStreamSynchronize(c->st));
      for (int64_t p = 0; p < Kg; ++p)
        if (og[p].status == 0 && og[p].n_points > 0) finish_network(og[p], ijs[(size_t)p]);
      auto t1 = std::chrono::steady_clock::now();
      double d2h = std::chrono::duration<double, std::milli>(t1 - t0).count();
      if (want_flow) {
        unsigned hw = std::max(1u, std::thread::hardware_concurrency());
        unsigned nt = (unsigned)std::min<int64_t>(Kg, std::min(hw, 16u));
        std::atomic<int64_t> next{0};
        auto worker = [&]() {
          for (;;) {
            int64_t p = next.fetch_add(1);
            if (p >= Kg) break;
            if (og[p].status == 0 && og[p].n_points > 0) solve_flow(og[p], o.pivot_cap);
          }
        };
        std::vector<std::thread> th;
        for (unsigned i = 1; i < nt; ++i) th.emplace_back(worker);
        worker();
        for (auto& t : th) t.join();
      }
      auto t2 = std::chrono::steady_clock::now();
      double fl = std::chrono::duration<double, std::milli>(t2 - t1).count();
      for (int64_t p = 0; p < Kg; ++p) {
        og[p].t_ms[W1_T_D2H] = d2h;
        og[p].t_ms[W1_T_FLOW] = fl;
        if (!keep) free_network(og[p]);
      }
    }
    return W1_OK;
  } catch (const StageError& e) {
    (void)hipGetLastError();
    (void)hipStreamSynchronize((hipStream_t)stream);
    if (out)
      for (int64_t p = 0; p < K; ++p) {
        w1_result_free(&out[p]);
        std::memset(&out[p], 0, sizeof(w1_result));
        out[p].status = e.code;
      }
    return e.code;
  } catch (const std::bad_alloc&) {
    return W1_ENOMEM;
  }
}

}  // namespace
}  // namespace w1

// ------------------------------------------------ allocation-free scratch --
// Device scratch of the allocation-free RWMD entry point: one fixed array per
// GPU, held for the life of the process.  In host code `scratch` names only a
// host-side stand-in; its device address comes from hipGetSymbolAddress, once
// per device with that device current, and only that address is used.
static __device__ __align__(256) char scratch[w1::kNoAllocScratchBytes];

namespace w1 {
namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};

// Device address of `scratch` on `device` (which must be current).
int scratch_setup(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return W1_ENODEV;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[device]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return W1_EHIP;
    }
    g_scratch_addr[device] = ptr;
  }
  *out = g_scratch_addr[device];
  return W1_OK;
}

}  // namespace
}  // namespace w1

// =========================================================================== ABI
using namespace w1;


extern "C" {

int w1_ctx_create(int device, w1_ctx** out) {
  if (!out) return W1_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
    (void)hipGetLastError();
    return W1_ENODEV;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return W1_ENODEV;
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return W1_ENODEV;
  w1_ctx* c = new (std::nothrow) w1_ctx();
  if (!c) return W1_ENOMEM;
  c->device = device;
  c->num_cus = prop.multiProcessorCount;
  c->trace = std::getenv("W1_TRACE") != nullptr;
  if (hipSetDevice(device) != hipSuccess || hipHostMalloc((void**)&c->hpin, 4096, hipHostMallocDefault) != hipSuccess) {
    delete c;
    return W1_EHIP;
  }
  for (int i = 0; i < 11; ++i)
    if (hipEventCreate(&c->kev[i]) != hipSuccess) {
      delete c;
      return W1_EHIP;
    }
  for (int i = 0; i < 8; ++i)
    if (hipEventCreate(&c->ev[i]) != hipSuccess) {
      delete c;
      return W1_EHIP;
    }
  const int rc = scratch_setup(device, &c->scratch);
  if (rc != W1_OK) {
    w1_ctx_destroy(c);
    return rc;
  }
  *out = c;
  return W1_OK;
}

int w1_ctx_destroy(w1_ctx* c) {
  if (!c) return W1_EINVAL;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  for (DBuf* b : c->all)
    if (b->p) (void)hipFree(b->p);
  for (int i = 0; i < 8; ++i) (void)hipEventDestroy(c->ev[i]);
  for (int i = 0; i < 11; ++i) (void)hipEventDestroy(c->kev[i]);
  if (c->hpin) (void)hipHostFree(c->hpin);
  delete c;
  return W1_OK;
}

int w1_ctx_hip_error(const w1_ctx* c) { return c ? c->hip_err : 0; }

int w1_approx(w1_ctx* c, const w1_pd* a, const w1_pd* b, const w1_params* params, void* stream, w1_result* out) {
  return entry(c, a, b, 1, params, stream, out, nullptr);
}

int w1_approx_batch(w1_ctx* c, const w1_pd* a, const w1_pd* b, int64_t k, const w1_params* params, void* stream,
                    w1_result* out) {
  return entry(c, a, b, k, params, stream, out, nullptr);
}

int w1_rwmd(w1_ctx* c, const w1_pd* a, const w1_pd* b, int64_t k, uint32_t flags, void* stream, double* L_out) {
  if (!L_out) return W1_EINVAL;
  w1_params p{0.1, 0.1, 0, flags, 0};
  return entry(c, a, b, k, &p, stream, nullptr, L_out);
}

int w1_rwmd_noalloc(w1_ctx* c, const w1_pd* a, const w1_pd* b, int64_t k, uint32_t flags, void* stream,
                    double* L_out) {
  if (!c || !a || !b || k <= 0 || !L_out || (flags & ~(W1_INPUT_DEVICE | W1_METRIC_L2))) return W1_EINVAL;
  if (k > kNoAllocMaxPairs) return W1_ERANGE;
  int64_t total = 0;
  for (int64_t p = 0; p < k; ++p) {
    if (a[p].n < 0 || b[p].n < 0) return W1_EINVAL;
    total += a[p].n + b[p].n;
    if (total > kNoAllocMaxPoints) return W1_ERANGE;
  }
  if (!c->scratch) return W1_ENODEV;
  if (hipSetDevice(c->device) != hipSuccess) return W1_EHIP;
  // put the context's own buffers aside: every buffer of this call is a
  // slice of the device's scratch array
  for (size_t i = 0; i < c->all.size(); ++i) {
    c->saved[i] = *c->all[i];
    *c->all[i] = DBuf{};
  }
  c->arena = Arena{(char*)c->scratch, kNoAllocScratchBytes, 0};
  Opts o;
  o.flags = flags;
  int rc;
  try {
    c->K_base = 0;
    rc = run(*c, a, b, k, o, (hipStream_t)stream, nullptr, L_out);
  } catch (const StageError& e) {
    (void)hipGetLastError();
    (void)hipStreamSynchronize((hipStream_t)stream);
    rc = e.code;
  } catch (const std::bad_alloc&) {
    rc = W1_ENOMEM;
  }
  c->arena = Arena{};
  for (size_t i = 0; i < c->all.size(); ++i) *c->all[i] = c->saved[i];
  c->network_valid = false;
  return rc;
}

int w1_device_network_get(w1_ctx* c, int64_t k, w1_device_network* out) {
  if (!c || !out || !c->network_valid) return W1_EINVAL;
  k -= c->K_base;
  if (k < 0 || k >= c->K) return W1_EINVAL;
  const int64_t cs = c->h_cell_start[(size_t)k], as = c->h_arc_start[(size_t)k];
  out->n_cells = c->h_ncells[(size_t)k];
  out->n_pairs = c->h_npairs[(size_t)k];
  out->n_arcs = c->h_narcs[(size_t)k];
  out->cell_ij = (const int32_t*)c->cij.p + 2 * cs;
  out->cell_ca = (const int32_t*)c->ca.p + cs;
  out->cell_cb = (const int32_t*)c->cb.p + cs;
  out->supply = (const int64_t*)c->supply.p + cs + 2 * k;
  out->row_ptr = (const int64_t*)c->rp.p + cs + 3 * k;
  out->col = (const uint32_t*)c->l1.p + as;
  out->cost = c->network_l2 ? nullptr : (const int32_t*)c->costb.p + as;
  out->cost64 = c->network_l2 ? (const int64_t*)c->costb.p + as : nullptr;
  return W1_OK;
}

int w1_ctx_get_tuning(const w1_ctx* c, w1_tuning* out) {
  if (!c || !out) return W1_EINVAL;
  out->stack_depth = c->tun.stack_depth;
  out->work_cap = c->tun.work_cap;
  out->chunk_items = c->tun.chunk_items;
  out->blocks_per_cu = c->tun.blocks_per_cu;
  out->max_points_per_launch = c->max_points;
  out->compact_records = c->tun.compact;
  out->stream_max_rounds = c->stream_rounds;
  out->stream_graph = c->stream_graph;
  out->stream_arena_pairs = c->stream_arena;
  out->blocked_emit = c->blocked_emit;
  out->sort_window_words = c->sort_window;
  out->emit_block_limit = c->emit_block_limit;
  out->fused_expand_cells = c->fused_expand_cells;
  out->fused_expand_items = c->fused_expand_items;
  return W1_OK;
}

int w1_ctx_set_tuning(w1_ctx* c, const w1_tuning* t) {
  if (!c || !t) return W1_EINVAL;
  if (t->stack_depth < 8 || t->stack_depth > 32 || t->work_cap < 1 || t->work_cap > (1 << 20) ||
      t->chunk_items < 1 || t->chunk_items > (1 << 20) || t->blocks_per_cu < 1 || t->blocks_per_cu > 16 ||
      t->max_points_per_launch < 1 || (t->compact_records != 0 && t->compact_records != 1) ||
      t->stream_max_rounds < 0 || t->stream_arena_pairs < 0 || t->stream_arena_pairs > (int64_t(1) << 36) ||
      (t->blocked_emit != 0 && t->blocked_emit != 1) || t->sort_window_words < 0 || t->emit_block_limit < 0 ||
      t->fused_expand_cells < 0 || t->fused_expand_cells > kFusedExpandMaxCells || t->fused_expand_items < 0 ||
      (t->stream_graph != 0 && t->stream_graph != 1))
    return W1_EINVAL;
  c->tun = WspdTuning{t->stack_depth, t->work_cap, t->chunk_items, t->blocks_per_cu, t->compact_records};
  c->max_points = t->max_points_per_launch;
  c->stream_rounds = t->stream_max_rounds;
  c->stream_graph = t->stream_graph;
  c->stream_arena = t->stream_arena_pairs;
  c->blocked_emit = t->blocked_emit;
  c->emit_block_limit = t->emit_block_limit;
  c->sort_window = t->sort_window_words;
  c->fused_expand_cells = t->fused_expand_cells;
  c->fused_expand_items = t->fused_expand_items;
  return W1_OK;
}

int w1_ctx_last_kernel_times(const w1_ctx* c, double* ms, int n) {
  if (!c || !ms || n < 4) return W1_EINVAL;
  for (int i = 0; i < n; ++i) ms[i] = i < kNumKernelTimes ? c->kms[i] : 0.0;
  return W1_OK;
}

int w1_flow_solve(int64_t n_nodes, int64_t m, const uint32_t* src, const uint32_t* dst, const int32_t* cost,
                  const int64_t* supply, int64_t pivot_cap, int64_t* cost_out, int64_t* flow_out, int64_t* pot_out,
                  int64_t* pivots_out, int32_t* status_out) {
  if (n_nodes < 0 || m < 0 || (m > 0 && (!src || !dst || !cost)) || (n_nodes > 0 && !supply) || !cost_out)
    return W1_EINVAL;
  FlowResult fr{};
  fr.flow = flow_out;
  fr.pot = pot_out;
  int rc;
  try {
    rc = network_simplex_arcs(n_nodes, m, src, dst, cost, supply, pivot_cap, &fr);
  } catch (const std::bad_alloc&) {
    return W1_ENOMEM;
  }
  if (rc == -3) return W1_ENOMEM;
  if (rc != 0) return W1_EINVAL;
  *cost_out = fr.cost;  // -1 after a stall that left supply unrouted
  if (pivots_out) *pivots_out = fr.pivots;
  if (status_out) *status_out = fr.status ? W1_STALLED : W1_OPTIMAL;
  return W1_OK;
}

int w1_separation_for_eps(double eps, double kappa) {
  if (kappa <= 0) kappa = 0.1;
  if (!(eps > 0.0 && eps <= 1.0) || !(kappa < 0.5)) return W1_EINVAL;
  return separation(eps, kappa);
}

void w1_result_free(w1_result* r) {
  if (!r) return;
  free_network(*r);
  void* ptrs[] = {r->loc_b, r->loc_d, r->loc_w, r->loc_t, r->node_lo, r->node_hi, r->node_left, r->node_right,
                  r->node_box};
  for (void* q : ptrs) std::free(q);
  r->loc_b = r->loc_d = r->loc_t = nullptr;
  r->loc_w = nullptr;
  r->node_lo = r->node_hi = r->node_left = r->node_right = r->node_box = nullptr;
}

const char* w1_strerror(int code) {
  switch (code) {
    case W1_OK: return "ok";
    case W1_EINVAL: return "invalid argument or diagram point";
    case W1_ERANGE: return "grid extent or coordinate range exceeded";
    case W1_ENOMEM: return "out of memory";
    case W1_EHIP: return "HIP runtime error";
    case W1_EOVERFLOW: return "internal work list capacity exceeded";
    case W1_ENODEV: return "no gfx950 device";
  }
  return "unknown error";
}

}  // extern "C"
