// Library context: device buffers that persist between calls, the stream of
// the current call, events, and small helpers shared by the host code.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <initializer_list>
#include <vector>

#include "../../include/w1approx.h"
#include "common.h"
#include "kernels.h"

namespace w1 {

struct DBuf {
  void* p = nullptr;
  size_t cap = 0;
};

struct StageError {
  int code;
};

// A fixed device region that replaces allocation for one call: while a
// context has an arena, need() hands out consecutive 256-byte aligned slices
// of it and never calls hipMalloc; running past its end is W1_EOVERFLOW.
struct Arena {
  char* base = nullptr;
  size_t cap = 0, off = 0;
};

// Limits of the allocation-free RWMD entry point (w1_rwmd_noalloc): its
// device scratch, and the host tables it uses instead of growable ones.
constexpr size_t kNoAllocScratchBytes = size_t(128) << 20;
constexpr int64_t kNoAllocMaxPoints = int64_t(1) << 19;
constexpr int64_t kNoAllocMaxPairs = 1024;

// w1_ctx_last_kernel_times: work list, count pass, emit pass, pairs emitted,
// then the network passes: bucket histogram, bucket scatter, row histogram,
// row scatter (with the degree scan), row sort (with the diagonal rows).
constexpr int kNumKernelTimes = 12;

// Blocked emission of a single pair's network: used from this many
// work-list chunks on, sized by a count over every kSampleStride-th chunk.
constexpr int64_t kBlockedMinChunks = 4096;
constexpr int kSampleStride = 16;

struct Ctx {
  int device = 0;
  int num_cus = 256;
  int hip_err = 0;
  bool trace = false;
  hipStream_t st = nullptr;
  uint64_t* hpin = nullptr;  // pinned host scratch for read-backs
  WspdTuning tun{16, 1024, 512, 5, 1};
  int64_t max_points = int64_t(1) << 22;  // points per launch group of a batch
  int64_t stream_arena = 0;                // streamed emission: arena capacity in pair records (0 = off)
  int32_t stream_rounds = 0;               // streamed emission: arena fills at most (0 = all)
  int32_t stream_graph = 1;                // streamed emission: arena fills replayed from one captured graph
  int32_t fused_expand_cells = 4096;       // work-list expansion in one workgroup up to this many cells
  int32_t fused_expand_items = 0;          // its room in items (0: from the cell count)
  int32_t blocked_emit = 0;                // network path: blocked emission (off by default)
  int64_t emit_block_limit = 0;            // blocked emission: block cap (0 = as sized)
  int32_t sort_window = 0;                 // row sort bitmap window in words (0 = automatic)
  int64_t K_base = 0;                      // first pair of the last launch group
  std::vector<DBuf*> all;
  // points
  DBuf stage, orpart, segs, pb, pd, psd, kw0, kw1, kw2, kA, kB, vA, vB, head, idx, scantmp, sorttmp, small;
  // groups / locations
  DBuf gb, gd, gpair, gw, lb, ld, lw, lpair, lt, lterm, lbin, li, lj;
  // rwmd buckets
  DBuf nbuck, bincnt, binstart, ent, entl;
  // cells / tree
  DBuf ckey, cpair, cij, ca, cb, iaux, ibox, iheight, iparent, ndepth, inode, rmap, isplit;
  // wspd
  DBuf itemsA, itemsB, itemsX, itemsI, itemsS, icnt, ipos, ipp, cid, pcap, cfirst, cend, cpairs, ccnt, coff, xrange, xctr, err;
  // network: pu holds the 12-byte WSPD pair records (u, v, cost) and later
  // the unsorted row heads; l1 the bucket-major arc entries and later the
  // sorted heads (col); costb the arc costs; rp the per-pair row pointers
  DBuf pu, l1, costb, rp, supply, rstart, bcnt, bstart, tfirst, bcur, rowcnt, rowcur, bflag, bpos, deg, off, parc;
  // streamed emission: per-chunk pair checksums; Euclidean cost scale
  DBuf csum, pxmax, runxr, runbase, pslot, rowq;
  // blocked emission (network path): block fills, block pairs, counters;
  // blocks used by the last launch group (0: counted layout) and their size
  DBuf bfill, bpairs, bctl;
  uint32_t emit_blocks = 0, emit_block_recs = 0;
  int rec_words = 3;  // words per pair record of the last emit pass: (u, v) or (u, v, cost)
  // per pair
  DBuf pairs;
  int64_t pair_bytes = 0;  // bytes of the per-pair arrays in `pairs`
  PairArrays P{};
  int64_t K = 0;
  std::vector<int64_t> h_cell_start, h_ncells, h_npairs, h_arc_start, h_narcs;
  bool network_valid = false;
  bool network_l2 = false;  // the last network has 64-bit (Euclidean) costs
  hipEvent_t ev[8];
  hipEvent_t kev[11];  // WSPD work list, count, emit; network passes
  double kms[kNumKernelTimes] = {0};
  // allocation-free calls: the device's scratch region (set up when the
  // context is created), the arena carved from it during such a call, the
  // context's own buffers put aside meanwhile, and fixed host tables
  void* scratch = nullptr;
  Arena arena;
  std::vector<DBuf> saved;
  SegDesc seg_fixed[2 * kNoAllocMaxPairs];
  int32_t err_fixed[kNoAllocMaxPairs];

  Ctx() {
    DBuf* list[] = {&stage, &orpart, &segs, &pb, &pd, &psd, &kw0, &kw1, &kw2, &kA, &kB, &vA, &vB, &head, &idx, &scantmp, &sorttmp,
                    &small, &gb, &gd, &gpair, &gw, &lb, &ld, &lw, &lpair, &lt, &lterm, &lbin, &li, &lj, &nbuck,
                    &bincnt, &binstart, &ent, &entl, &ckey, &cpair, &cij, &ca, &cb, &iaux, &ibox, &iheight, &iparent,
                    &ndepth, &inode, &rmap, &isplit, &itemsA, &itemsB, &itemsX, &itemsI, &itemsS, &icnt, &ipos, &ipp, &cid, &pcap,
                    &cfirst, &cend, &cpairs, &ccnt, &coff, &xrange, &xctr, &err, &pu, &l1, &costb, &rp,
                    &supply, &rstart, &bcnt, &bstart, &tfirst, &bcur, &rowcnt, &rowcur, &bflag, &bpos, &deg, &off,
                    &parc, &csum, &pxmax, &runxr, &runbase, &pslot, &rowq, &pairs};
    all.assign(std::begin(list), std::end(list));
    saved.resize(all.size());
  }
};

inline void check(Ctx& c, hipError_t e) {
  if (e != hipSuccess) {
    c.hip_err = (int)e;
    throw StageError{W1_EHIP};
  }
}

template <typename T>
T* need(Ctx& c, DBuf& b, int64_t count) {
  size_t bytes = (size_t)std::max<int64_t>(count, 1) * sizeof(T);
  bytes = (bytes + 255) & ~(size_t)255;
  if (c.arena.base) {  // allocation-free call: every buffer is a slice of the arena
    if (b.p && bytes <= b.cap) return (T*)b.p;
    if (bytes > c.arena.cap - c.arena.off) throw StageError{W1_EOVERFLOW};
    b.p = c.arena.base + c.arena.off;
    b.cap = bytes;
    c.arena.off += bytes;
    return (T*)b.p;
  }
  if (bytes > b.cap) {
    if (b.p) {
      check(c, hipStreamSynchronize(c.st));
      (void)hipFree(b.p);
      b.p = nullptr;
      b.cap = 0;
    }
    size_t want = std::max(bytes, b.cap + b.cap / 2);
    if (hipMalloc(&b.p, want) != hipSuccess) {
      (void)hipGetLastError();
      if (hipMalloc(&b.p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        b.p = nullptr;
        throw StageError{W1_ENOMEM};
      }
      want = bytes;
    }
    b.cap = want;
  }
  return (T*)b.p;
}

// Grow while keeping the first `keep` elements.
template <typename T>
T* grow_keep(Ctx& c, DBuf& b, int64_t count, int64_t keep) {
  size_t bytes = (size_t)std::max<int64_t>(count, 1) * sizeof(T);
  if (bytes <= b.cap) return (T*)b.p;
  DBuf nb;
  T* np = need<T>(c, nb, count * 2);
  if (keep > 0) check(c, hipMemcpyAsync(np, b.p, (size_t)keep * sizeof(T), hipMemcpyDeviceToDevice, c.st));
  check(c, hipStreamSynchronize(c.st));
  if (b.p && !c.arena.base) (void)hipFree(b.p);
  b = nb;
  return np;
}

template <typename T>
inline void readback(Ctx& c, const T* dev, T* host, int64_t count) {
  if (count <= 0) return;
  check(c, hipMemcpyAsync(host, dev, (size_t)count * sizeof(T), hipMemcpyDeviceToHost, c.st));
  check(c, hipStreamSynchronize(c.st));
}

// Small host -> device copy that completes before returning (the host
// buffer may be released right after).
inline void upload(Ctx& c, void* dev, const void* host, size_t bytes) {
  if (!bytes) return;
  check(c, hipMemcpyAsync(dev, host, bytes, hipMemcpyHostToDevice, c.st));
  check(c, hipStreamSynchronize(c.st));
}

// Several small host -> device copies with one wait for all of them.
struct HostCopy {
  void* dev;
  const void* host;
  size_t bytes;
};
inline void upload_all(Ctx& c, std::initializer_list<HostCopy> copies) {
  bool any = false;
  for (const HostCopy& x : copies)
    if (x.bytes) {
      check(c, hipMemcpyAsync(x.dev, x.host, x.bytes, hipMemcpyHostToDevice, c.st));
      any = true;
    }
  if (any) check(c, hipStreamSynchronize(c.st));
}

inline uint64_t read_u64(Ctx& c, const void* dev) {
  check(c, hipMemcpyAsync(c.hpin, dev, 8, hipMemcpyDeviceToHost, c.st));
  check(c, hipStreamSynchronize(c.st));
  return c.hpin[0];
}

}  // namespace w1

struct w1_ctx : w1::Ctx {};
