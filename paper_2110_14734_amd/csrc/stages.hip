// Stage kernels of the approximate W1 pipeline (all but the WSPD traversal).
//
//   a0  load + validate + 0-condensation of A u B with net multiplicities
//       (Sec. 4.3; co-located A and B points merge with added supplies, the
//       overlap rule of Sec. 5.3 at delta = 0)
//   a1  RWMD lower bound (Alg. 1, diagonal arc included) on a uniform bucket
//       grid, exact int64 fixed-point sum
//   a2  delta-condensation onto the power-of-two grid (Alg. 2, k = 1, no
//       jitter) and Morton ordering of the cells
//   a3  binary radix tree over (pair, Morton) keys with tight boxes
//   a5  diagonal arcs (Alg. 7), the B-to-A diagonal arc, supplies
//
// Every kernel handles a batch of diagram pairs at once: points, locations
// and cells are sorted by pair first, so a pair's data is contiguous and
// per-pair scalars live in PairArrays.  All arithmetic that decides a
// discrete outcome (RWMD terms, grid cells, keys) is IEEE FP64 or integer
// and order-independent, so results are bit-identical run to run.
#include "common.h"
#include "kernels.h"

namespace w1 {

namespace {

__device__ inline int64_t ld_i64(const int64_t* p) { return *p; }

template <typename T>
__device__ inline T op_add(T a, T b) { return a + b; }

__device__ inline uint64_t u64max(uint64_t a, uint64_t b) { return a > b ? a : b; }
__device__ inline uint64_t u64min(uint64_t a, uint64_t b) { return a < b ? a : b; }

__device__ inline void set_err(int32_t* err, int32_t code) { atomicMin(err, code); }

__device__ inline int bitlen64(uint64_t k) { return k ? 64 - __clzll((long long)k) : 0; }

// Spread the low 30 bits of v to the even bit positions of a 60-bit word.
__device__ inline uint64_t spread30(uint64_t v) {
  uint64_t x = v & 0x3fffffffull;
  x = (x | (x << 16)) & 0x0000FFFF0000FFFFull;
  x = (x | (x << 8)) & 0x00FF00FF00FF00FFull;
  x = (x | (x << 4)) & 0x0F0F0F0F0F0F0F0Full;
  x = (x | (x << 2)) & 0x3333333333333333ull;
  x = (x | (x << 1)) & 0x5555555555555555ull;
  return x;
}

// ===================================================================== a0 ==
__global__ void k_load(const SegDesc* __restrict__ segs, int nseg, int64_t total, int dtype, double* __restrict__ pb,
                       double* __restrict__ pd, uint32_t* __restrict__ psd, uint64_t* __restrict__ kw0,
                       uint64_t* __restrict__ kw1, uint64_t* __restrict__ kw2, int32_t* __restrict__ perr) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= total) return;
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (segs[mid].out_off <= x) lo = mid;
    else hi = mid - 1;
  }
  const SegDesc sg = segs[lo];
  const int64_t k = x - sg.out_off;
  double b, d;
  if (dtype == 0) {
    const float* p = (const float*)sg.ptr;
    b = (double)p[2 * k];
    d = (double)p[2 * k + 1];
  } else {
    const double* p = (const double*)sg.ptr;
    b = p[2 * k];
    d = p[2 * k + 1];
  }
  b = b + 0.0;  // fold -0.0 into +0.0 so equal values have equal bits
  d = d + 0.0;
  bool bad = !(isfinite(b) && isfinite(d)) || d < b;
  if (bad) set_err(&perr[sg.pair], -1);
  const bool drop = bad || d == b;
  pb[x] = b;
  pd[x] = d;
  psd[x] = ((uint32_t)sg.pair << 1) | (uint32_t)sg.side;
  kw0[x] = ordered_bits(dbl_bits(d));
  kw1[x] = ordered_bits(dbl_bits(b));
  kw2[x] = ((uint64_t)drop << 40) | (uint64_t)sg.pair;
}

// After sorting the points by (drop, pair, birth, death): a point opens a
// group when any of those differ from its predecessor.
__global__ void k_group_heads(const uint32_t* __restrict__ perm, const uint64_t* __restrict__ kw2s,
                              const double* __restrict__ pb, const double* __restrict__ pd, int64_t n,
                              uint32_t* __restrict__ head) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  uint32_t h = 0;
  if (!(kw2s[k] >> 40)) {
    if (k == 0) h = 1;
    else {
      uint32_t a = perm[k], q = perm[k - 1];
      h = (kw2s[k] != kw2s[k - 1] || pb[a] != pb[q] || pd[a] != pd[q]) ? 1u : 0u;
    }
  }
  head[k] = h;
}

__global__ void k_group_fill(const uint32_t* __restrict__ perm, const uint64_t* __restrict__ kw2s,
                             const uint32_t* __restrict__ head, const uint32_t* __restrict__ gidx,
                             const double* __restrict__ pb, const double* __restrict__ pd, const uint32_t* __restrict__ psd,
                             int64_t n, double* __restrict__ gb, double* __restrict__ gd, uint32_t* __restrict__ gpair,
                             int32_t* __restrict__ gw) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool valid = k < n && !(kw2s[k] >> 40);
  uint32_t g = ~0u;
  int32_t w = 0;
  if (valid) {
    g = gidx[k] + head[k] - 1;
    uint32_t a = perm[k];
    uint32_t sd = psd[a];
    w = (sd & 1u) ? -1 : 1;
    if (head[k]) {
      gb[g] = pb[a];
      gd[g] = pd[a];
      gpair[g] = sd >> 1;
    }
  }
  if (wave_seg_reduce(g, w, op_add<int32_t>)) atomicAdd(&gw[g], w);
}

__global__ void k_count_total(const uint32_t* __restrict__ head, const uint32_t* __restrict__ scanned, int64_t n,
                              uint64_t* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *out = n > 0 ? (uint64_t)scanned[n - 1] + head[n - 1] : 0;
}

__global__ void k_count_total64(const uint64_t* __restrict__ cnt, const uint64_t* __restrict__ scanned, int64_t n,
                                uint64_t* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *out = n > 0 ? scanned[n - 1] + cnt[n - 1] : 0;
}

__global__ void k_nonzero_flags(const int32_t* __restrict__ gw, int64_t G, uint32_t* __restrict__ flag) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < G) flag[g] = gw[g] != 0 ? 1u : 0u;
}

__global__ void k_loc_fill(const int32_t* __restrict__ gw, const uint32_t* __restrict__ flag,
                           const uint32_t* __restrict__ lidx, const double* __restrict__ gb, const double* __restrict__ gd,
                           const uint32_t* __restrict__ gpair, int64_t G, double* __restrict__ lb, double* __restrict__ ld,
                           int32_t* __restrict__ lw, uint32_t* __restrict__ lpair, PairArrays P) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t key = ~0u;
  int64_t na = 0, nb = 0;
  int32_t ca = 0, cb = 0;
  if (g < G && flag[g]) {
    uint32_t l = lidx[g];
    int32_t w = gw[g];
    lb[l] = gb[g];
    ld[l] = gd[g];
    lw[l] = w;
    key = gpair[g];
    lpair[l] = key;
    if (w > 0) { na = w; ca = 1; }
    else { nb = -(int64_t)w; cb = 1; }
  }
  const uint32_t k0 = key;
  const bool one = block_single_key(k0);
  bool t = wave_seg_reduce(k0, na, op_add<int64_t>);
  wave_seg_reduce(k0, nb, op_add<int64_t>);
  wave_seg_reduce(k0, ca, op_add<int32_t>);
  wave_seg_reduce(k0, cb, op_add<int32_t>);
  if (one) {
    na = block_total(na, op_add<int64_t>);
    nb = block_total(nb, op_add<int64_t>);
    ca = block_total(ca, op_add<int32_t>);
    cb = block_total(cb, op_add<int32_t>);
    t = threadIdx.x == 0;
  }
  if (t) {
    if (na) atomicAdd((unsigned long long*)&P.nA[k0], (unsigned long long)na);
    if (nb) atomicAdd((unsigned long long*)&P.nB[k0], (unsigned long long)nb);
    if (ca) atomicAdd(&P.locA[k0], ca);
    if (cb) atomicAdd(&P.locB[k0], cb);
  }
}

// ===================================================================== a1 ==
__global__ void k_loc_bbox(const double* __restrict__ lb, const double* __restrict__ ld, const uint32_t* __restrict__ lpair,
                           int64_t M, PairArrays P) {
  const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t key = ~0u;
  uint64_t b0 = ~0ull, b1 = 0, d0 = ~0ull, d1 = 0;
  if (l < M) {
    key = lpair[l];
    b0 = b1 = ordered_bits(dbl_bits(lb[l]));
    d0 = d1 = ordered_bits(dbl_bits(ld[l]));
  }
  const bool one = block_single_key(key);
  bool t = wave_seg_reduce(key, b0, u64min);
  wave_seg_reduce(key, b1, u64max);
  wave_seg_reduce(key, d0, u64min);
  wave_seg_reduce(key, d1, u64max);
  if (one) {
    b0 = block_total(b0, u64min);
    b1 = block_total(b1, u64max);
    d0 = block_total(d0, u64min);
    d1 = block_total(d1, u64max);
    t = threadIdx.x == 0;
  }
  if (t) {
    atomicMin((unsigned long long*)&P.bmin[key], (unsigned long long)b0);
    atomicMax((unsigned long long*)&P.bmax[key], (unsigned long long)b1);
    atomicMin((unsigned long long*)&P.dmin[key], (unsigned long long)d0);
    atomicMax((unsigned long long*)&P.dmax[key], (unsigned long long)d1);
  }
}

// Bucket grid of one pair: side h = 2^beh with h >= extent / sqrt(#locations)
// so the grid has at most about #locations + 4 sqrt(#locations) + 4 buckets.
// Any side gives the same (exact) nearest neighbours; this one keeps the
// grid proportional to the data.
__global__ void k_bucket_setup(PairArrays P, int64_t K, int64_t* __restrict__ nbuckets) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= K) return;
  const int64_t m = (int64_t)P.locA[p] + P.locB[p];
  P.bnx[p] = P.bny[p] = 0;
  P.beh[p] = 0;
  P.bx0[p] = P.by0[p] = 0;
  nbuckets[p] = 0;
  if (m == 0 || P.err[p]) return;
  const double b0 = ordered_to_dbl(P.bmin[p]), b1 = ordered_to_dbl(P.bmax[p]);
  const double d0 = ordered_to_dbl(P.dmin[p]), d1 = ordered_to_dbl(P.dmax[p]);
  double S = fmax(b1 - b0, d1 - d0);
  double target = S / sqrt((double)m);
  if (!(target > 0.0)) target = fmax(fmax(fabs(b0), fabs(b1)), fmax(fabs(d0), fabs(d1)));
  if (!(target > 0.0)) target = 1.0;
  int E = 0;
  frexp(target, &E);
  const double x0 = floor(ldexp(b0, -E)), x1 = floor(ldexp(b1, -E));
  const double y0 = floor(ldexp(d0, -E)), y1 = floor(ldexp(d1, -E));
  const double lim = 0x1p52;
  if (!(fabs(x0) < lim && fabs(x1) < lim && fabs(y0) < lim && fabs(y1) < lim)) {
    set_err(&P.err[p], -2);
    return;
  }
  const int64_t nx = (int64_t)x1 - (int64_t)x0 + 1, ny = (int64_t)y1 - (int64_t)y0 + 1;
  P.beh[p] = E;
  P.bx0[p] = (int64_t)x0;
  P.by0[p] = (int64_t)y0;
  P.bnx[p] = (int32_t)nx;
  P.bny[p] = (int32_t)ny;
  nbuckets[p] = nx * ny;
}

__device__ inline void bucket_of(const PairArrays& P, uint32_t p, double b, double d, int64_t* ix, int64_t* iy) {
  const int E = P.beh[p];
  *ix = (int64_t)floor(ldexp(b, -E)) - P.bx0[p];
  *iy = (int64_t)floor(ldexp(d, -E)) - P.by0[p];
}

__global__ void k_bucket_count(const double* __restrict__ lb, const double* __restrict__ ld, const int32_t* __restrict__ lw,
                               const uint32_t* __restrict__ lpair, int64_t M, PairArrays P, uint32_t* __restrict__ bincnt,
                               int64_t* __restrict__ lbin) {
  const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= M) return;
  const uint32_t p = lpair[l];
  if (P.err[p]) {
    lbin[l] = -1;
    return;
  }
  int64_t ix, iy;
  bucket_of(P, p, lb[l], ld[l], &ix, &iy);
  const int64_t bin = 2 * (P.bbase[p] + iy * P.bnx[p] + ix) + (lw[l] < 0 ? 1 : 0);
  lbin[l] = bin;
  atomicAdd(&bincnt[bin], 1u);
}

__global__ void k_bucket_fill(const double* __restrict__ lb, const double* __restrict__ ld, const int64_t* __restrict__ lbin,
                              int64_t M, const uint32_t* __restrict__ binstart, uint32_t* __restrict__ bincur,
                              double2* __restrict__ ent, uint32_t* __restrict__ entl) {
  const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= M) return;
  const int64_t bin = lbin[l];
  if (bin < 0) return;
  const uint32_t pos = binstart[bin] + atomicAdd(&bincur[bin], 1u);
  ent[pos] = make_double2(lb[l], ld[l]);
  entl[pos] = (uint32_t)l;
}

// Nearest location of the other diagram, capped by the cost to the diagonal.
// Metric of the nearest-neighbour search.  L-infinity: the running value is
// the distance itself, max(|db|, |dd|).  Euclidean: the running value is the
// squared distance q = db*db + dd*dd (each one IEEE double operation, in this
// order), and the cost is min(sqrt(q_min), (d - b) R) at the end, R the
// double nearest to 1/sqrt(2).  A location in ring r or beyond is at least
// r h away in L-infinity, hence in Euclidean distance too, and because r h
// is a double (h a power of two) its computed square and squared
// differences are at least (r h)^2: once q_min <= (r h)^2 no later location
// lowers it; once the diagonal cost is <= r h no later location can undercut
// it, its square root being at least r h.
constexpr double kRSqrt1_2 = 0x1.6a09e667f3bcdp-1;

template <bool L2>
struct NnMetric;

template <>
struct NnMetric<false> {
  __device__ static double start(double b, double d) { return 0.5 * (d - b); }
  __device__ static double eval(double b, double d, double qb, double qd) {
    const double dist = fabs(b - qb), dy = fabs(d - qd);
    return dy > dist ? dy : dist;
  }
  __device__ static bool done(double best, double diag, double rh) { return best <= rh; }
  __device__ static double finish(double best, double diag) { return best; }
  __device__ static double diag(double b, double d) { return 0.5 * (d - b); }
};

template <>
struct NnMetric<true> {
  __device__ static double start(double, double) { return __builtin_inf(); }
  __device__ static double eval(double b, double d, double qb, double qd) {
    const double gb = b - qb, gd = d - qd;
    return gb * gb + gd * gd;
  }
  __device__ static bool done(double best, double diag, double rh) { return best <= rh * rh || diag <= rh; }
  __device__ static double finish(double best, double diag) {
    const double t = sqrt(best);
    return t < diag ? t : diag;
  }
  __device__ static double diag(double b, double d) { return (d - b) * kRSqrt1_2; }
};

// Ring search over the other diagram's buckets: ring r holds the buckets at
// Chebyshev index distance r from the query's bucket; a location in ring r
// is at least (r - 1) h away (bucket indices are exact floors of
// power-of-two scalings), so after ring r nothing closer than r h remains.
template <bool L2>
struct RingSearch {
  const uint32_t* binstart;
  const double2* ent;
  int64_t base, nx, ny;
  int opp;
  __device__ void visit(int64_t x, int64_t y, double b, double d, double& best) const {
    const int64_t bin = 2 * (base + y * nx + x) + opp;
    const uint32_t e0 = binstart[bin], e1 = binstart[bin + 1];
    for (uint32_t e = e0; e < e1; ++e) {
      const double2 q = ent[e];
      const double v = NnMetric<L2>::eval(b, d, q.x, q.y);
      if (v < best) best = v;
    }
  }
  // rings r0, r0 + 1, ... until certified or past the grid
  __device__ void run(int64_t ix, int64_t iy, int64_t r0, int64_t rmax, double h, double b, double d, double diag,
                      double& best) const {
    for (int64_t r = r0;; ++r) {
      if (r == 0) {
        visit(ix, iy, b, d, best);
      } else {
        const int64_t x0 = ix - r < 0 ? 0 : ix - r, x1 = ix + r > nx - 1 ? nx - 1 : ix + r;
        const int64_t y0 = iy - r + 1 < 0 ? 0 : iy - r + 1, y1 = iy + r - 1 > ny - 1 ? ny - 1 : iy + r - 1;
        if (iy - r >= 0)
          for (int64_t x = x0; x <= x1; ++x) visit(x, iy - r, b, d, best);
        if (iy + r < ny)
          for (int64_t x = x0; x <= x1; ++x) visit(x, iy + r, b, d, best);
        if (ix - r >= 0)
          for (int64_t y = y0; y <= y1; ++y) visit(ix - r, y, b, d, best);
        if (ix + r < nx)
          for (int64_t y = y0; y <= y1; ++y) visit(ix + r, y, b, d, best);
      }
      if (NnMetric<L2>::done(best, diag, (double)r * h) || r >= rmax) break;
    }
  }
};

// Every location starts at its cost to the diagonal (locations of a pair
// with an error keep it).
template <bool L2>
__global__ void k_nn_init(const double* __restrict__ lb, const double* __restrict__ ld, const int32_t* __restrict__ lw,
                          int64_t M, double* __restrict__ lt, double* __restrict__ lterm) {
  const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= M) return;
  const double best = NnMetric<L2>::diag(lb[l], ld[l]);
  const int32_t w = lw[l];
  lt[l] = best;
  lterm[l] = (double)(w > 0 ? w : -w) * best;
}

// One wave per bucket side: the other diagram's locations in the 3x3 block
// of buckets around it (rings 0 and 1) are staged in LDS once and scanned by
// every query of the bucket.  Every location closer than h lies in that
// block, so a query certified at radius h is done; the others continue with
// ring 2 onwards.  A block with more candidates than fit runs the ring
// search from ring 0.  The minimum is over the same locations as the plain
// ring search, so the result is identical.
constexpr int kNnCand = 1024;

template <bool L2>
__global__ void __launch_bounds__(64) k_nn_bins(const int32_t* __restrict__ lw, const uint32_t* __restrict__ lpair,
                                                PairArrays P, const uint32_t* __restrict__ binstart,
                                                const double2* __restrict__ ent, const uint32_t* __restrict__ entl,
                                                double* __restrict__ lt, double* __restrict__ lterm) {
  __shared__ double2 cand[kNnCand];
  const int64_t qb = blockIdx.x;
  const uint32_t e0 = binstart[qb], e1 = binstart[qb + 1];
  if (e0 == e1) return;
  const int lane = lane_id();
  const uint32_t p = lpair[entl[e0]];  // every location of a bin belongs to one pair
  RingSearch<L2> rs{binstart, ent, P.bbase[p], P.bnx[p], P.bny[p], (int)(qb & 1) ^ 1};
  const int64_t cell = (qb >> 1) - rs.base;
  const int64_t ix = cell % rs.nx, iy = cell / rs.nx;
  int nc = 0;
  bool spill = false;
  for (int64_t y = iy - 1; y <= iy + 1; ++y)
    for (int64_t x = ix - 1; x <= ix + 1; ++x) {
      if (x < 0 || y < 0 || x >= rs.nx || y >= rs.ny) continue;
      const int64_t bin = 2 * (rs.base + y * rs.nx + x) + rs.opp;
      const uint32_t s0 = binstart[bin], cnt = binstart[bin + 1] - s0;
      if (nc + (int)cnt > kNnCand) {
        spill = true;
        continue;
      }
      for (uint32_t t = lane; t < cnt; t += WAVE) cand[nc + t] = ent[s0 + t];
      nc += (int)cnt;
    }
  __syncthreads();
  const double h = ldexp(1.0, P.beh[p]);
  int64_t rmax = ix;
  if (rs.nx - 1 - ix > rmax) rmax = rs.nx - 1 - ix;
  if (iy > rmax) rmax = iy;
  if (rs.ny - 1 - iy > rmax) rmax = rs.ny - 1 - iy;
  for (uint32_t e = e0 + lane; e < e1; e += WAVE) {
    const double2 me = ent[e];
    const double b = me.x, d = me.y;
    const double diag = NnMetric<L2>::diag(b, d);
    double best = NnMetric<L2>::start(b, d);
    if (spill) {
      rs.run(ix, iy, 0, rmax, h, b, d, diag, best);
    } else {
      for (int c = 0; c < nc; ++c) {
        const double2 q = cand[c];
        const double v = NnMetric<L2>::eval(b, d, q.x, q.y);
        if (v < best) best = v;
      }
      if (!NnMetric<L2>::done(best, diag, h) && rmax >= 2) rs.run(ix, iy, 2, rmax, h, b, d, diag, best);
    }
    const double t = NnMetric<L2>::finish(best, diag);
    const uint32_t l = entl[e];
    const int32_t w = lw[l];
    lt[l] = t;
    lterm[l] = (double)(w > 0 ? w : -w) * t;
  }
}

__global__ void k_term_max(const double* __restrict__ lterm, const int32_t* __restrict__ lw, const uint32_t* __restrict__ lpair,
                           int64_t M, PairArrays P) {
  const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t key = ~0u;
  uint64_t a = 0, b = 0;
  if (l < M) {
    key = lpair[l];
    uint64_t bits = dbl_bits(lterm[l]);  // non-negative: bit order = value order
    if (lw[l] > 0) a = bits;
    else b = bits;
  }
  const bool one = block_single_key(key);
  bool t = wave_seg_reduce(key, a, u64max);
  wave_seg_reduce(key, b, u64max);
  if (one) {
    a = block_total(a, u64max);
    b = block_total(b, u64max);
    t = threadIdx.x == 0;
  }
  if (t) {
    if (a) atomicMax((unsigned long long*)&P.tmaxA[key], (unsigned long long)a);
    if (b) atomicMax((unsigned long long*)&P.tmaxB[key], (unsigned long long)b);
  }
}

__device__ inline int32_t fixed_shift(uint64_t maxbits, int32_t count) {
  if (count == 0 || maxbits == 0) return 0;
  int E = 0;
  frexp(bits_dbl(maxbits), &E);
  return 62 - E - bitlen64((uint64_t)count);
}

__global__ void k_rwmd_shift(PairArrays P, int64_t K) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= K) return;
  P.FA[p] = fixed_shift(P.tmaxA[p], P.locA[p]);
  P.FB[p] = fixed_shift(P.tmaxB[p], P.locB[p]);
}

__global__ void k_term_sum(const double* __restrict__ lterm, const int32_t* __restrict__ lw, const uint32_t* __restrict__ lpair,
                           int64_t M, PairArrays P) {
  const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t key = ~0u;
  uint64_t a = 0, b = 0;
  if (l < M) {
    key = lpair[l];
    const bool isA = lw[l] > 0;
    const int32_t F = isA ? P.FA[key] : P.FB[key];
    const uint64_t q = (uint64_t)(int64_t)floor(ldexp(lterm[l], F));
    if (isA) a = q;
    else b = q;
  }
  const bool one = block_single_key(key);
  bool t = wave_seg_reduce(key, a, op_add<uint64_t>);
  wave_seg_reduce(key, b, op_add<uint64_t>);
  if (one) {
    a = block_total(a, op_add<uint64_t>);
    b = block_total(b, op_add<uint64_t>);
    t = threadIdx.x == 0;
  }
  if (t) {
    if (a) atomicAdd((unsigned long long*)&P.sumA[key], (unsigned long long)a);
    if (b) atomicAdd((unsigned long long*)&P.sumB[key], (unsigned long long)b);
  }
}

// L = max(L_A, L_B), each the fixed-point sum converted toward zero; grid
// exponent e with 2^e <= (1 - 2^-40) * 2 eps_c L / n (Prop. delta-
// condensation, L-infinity form: a point moves by at most g/2), times R for
// the Euclidean metric (a point moves by half a cell diagonal, g/sqrt(2)).
__global__ void k_params(PairArrays P, int64_t K, double eps_c, int l2) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= K) return;
  const int64_t n = P.nA[p] + P.nB[p];
  const int64_t SA = (int64_t)P.sumA[p], SB = (int64_t)P.sumB[p];
  const double LA = SA ? ldexp(__ll2double_rz(SA), -P.FA[p]) : 0.0;
  const double LB = SB ? ldexp(__ll2double_rz(SB), -P.FB[p]) : 0.0;
  const double L = LA > LB ? LA : LB;
  P.L[p] = L;
  P.e[p] = 0;
  if (n == 0 || P.err[p]) return;
  if (!(L > 0.0)) {
    set_err(&P.err[p], -2);
    return;
  }
  double gmax = ((2.0 * eps_c) * L) / (double)n;
  if (l2) gmax = gmax * kRSqrt1_2;
  const double gsafe = gmax * (1.0 - 0x1p-40);
  int E = 0;
  frexp(gsafe, &E);
  P.e[p] = E - 1;
}

// ===================================================================== a2 ==
__global__ void k_snap(const double* __restrict__ lb, const double* __restrict__ ld, const uint32_t* __restrict__ lpair,
                       int64_t M, PairArrays P, int64_t* __restrict__ li, int64_t* __restrict__ lj) {
  const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t key = ~0u;
  int64_t I = INT64_MAX;
  if (l < M) {
    const uint32_t p = lpair[l];
    if (!P.err[p]) {
      const int e = P.e[p];
      const double x = ldexp(lb[l], -e), y = ldexp(ld[l], -e);
      if (!(fabs(x) < 0x1p62 && fabs(y) < 0x1p62)) {
        set_err(&P.err[p], -2);
      } else {
        I = (int64_t)floor(x);
        li[l] = I;
        lj[l] = (int64_t)floor(y);
        key = p;
      }
    }
  }
  const auto imin = [](int64_t a, int64_t b) { return a < b ? a : b; };
  const bool one = block_single_key(key);
  bool t = wave_seg_reduce(key, I, imin);
  if (one) {
    I = block_total(I, imin);
    t = threadIdx.x == 0;
  }
  if (t) atomicMin((long long*)&P.m0[key], (long long)I);
}

__global__ void k_morton(const int64_t* __restrict__ li, const int64_t* __restrict__ lj, const uint32_t* __restrict__ lpair,
                         int64_t M, PairArrays P, uint64_t* __restrict__ kw0, uint64_t* __restrict__ kw1) {
  const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= M) return;
  const uint32_t p = lpair[l];
  uint64_t key = 0, hi = ((uint64_t)1 << 40) | p;
  if (!P.err[p]) {
    const int64_t i = li[l] - P.m0[p], j = lj[l] - P.m0[p];
    if (i >= ((int64_t)1 << 30) || j >= ((int64_t)1 << 30)) {
      set_err(&P.err[p], -2);
    } else {
      key = spread30((uint64_t)i) | (spread30((uint64_t)j) << 1);
      hi = p;
    }
  }
  kw0[l] = key;
  kw1[l] = hi;
}

__global__ void k_cell_heads(const uint32_t* __restrict__ perm, const uint64_t* __restrict__ kw1s,
                             const uint64_t* __restrict__ kw0, int64_t M, uint32_t* __restrict__ head) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= M) return;
  uint32_t h = 0;
  if (!(kw1s[k] >> 40)) {
    if (k == 0) h = 1;
    else h = (kw1s[k] != kw1s[k - 1] || kw0[perm[k]] != kw0[perm[k - 1]]) ? 1u : 0u;
  }
  head[k] = h;
}

__global__ void k_cell_fill(const uint32_t* __restrict__ perm, const uint64_t* __restrict__ kw1s,
                            const uint64_t* __restrict__ kw0, const uint32_t* __restrict__ head,
                            const uint32_t* __restrict__ cidx, const int64_t* __restrict__ li,
                            const int64_t* __restrict__ lj, const int32_t* __restrict__ lw, int64_t M, PairArrays P,
                            uint64_t* __restrict__ ckey, uint32_t* __restrict__ cpair, int2* __restrict__ cij,
                            int32_t* __restrict__ ca, int32_t* __restrict__ cb) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t c = ~0u;
  int32_t a = 0, b = 0;
  if (k < M && !(kw1s[k] >> 40)) {
    c = cidx[k] + head[k] - 1;
    const uint32_t l = perm[k];
    const uint32_t p = (uint32_t)kw1s[k];
    const int32_t w = lw[l];
    if (w > 0) a = w;
    else b = -w;
    if (head[k]) {
      ckey[c] = kw0[l];
      cpair[c] = p;
      cij[c] = make_int2((int)(li[l] - P.m0[p]), (int)(lj[l] - P.m0[p]));
    }
  }
  const uint32_t c0 = c;
  bool t = wave_seg_reduce(c0, a, op_add<int32_t>);
  wave_seg_reduce(c0, b, op_add<int32_t>);
  if (t) {
    if (a) atomicAdd(&ca[c0], a);
    if (b) atomicAdd(&cb[c0], b);
  }
}

// Bounds of each pair's run in a pair-major array of pair ids: the first
// element of a run writes lo[p], the last writes hi[p] (no atomics).
__global__ void k_run_bounds(const uint32_t* __restrict__ key, int64_t n, int64_t* __restrict__ lo,
                             int64_t* __restrict__ hi) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= n) return;
  const uint32_t p = key[x];
  if (x == 0 || key[x - 1] != p) lo[p] = x;
  if (x == n - 1 || key[x + 1] != p) hi[p] = x + 1;
}

__global__ void k_bounds_count32(const int64_t* __restrict__ lo, const int64_t* __restrict__ hi, int64_t K,
                                 int32_t* __restrict__ out) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < K) out[p] = (int32_t)(hi[p] - lo[p]);
}

// ===================================================================== a3 ==
__device__ inline int delta_pk(const uint32_t* __restrict__ cpair, const uint64_t* __restrict__ ckey, int64_t N,
                               int64_t i, int64_t j) {
  if (j < 0 || j >= N) return -1;
  const uint64_t pi = cpair[i], pj = cpair[j];
  if (pi != pj) return __clzll((long long)(pi ^ pj));
  return 64 + __clzll((long long)(ckey[i] ^ ckey[j]));
}

// Binary radix tree over sorted unique keys: internal node i covers a range
// with one end at i; the other end and the split are found by binary search
// on the common-prefix length.
__global__ void k_karras(const uint32_t* __restrict__ cpair, const uint64_t* __restrict__ ckey, int64_t N,
                         int4* __restrict__ iaux, int32_t* __restrict__ iparent) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N - 1) return;
  const int dn = delta_pk(cpair, ckey, N, i, i + 1), dp = delta_pk(cpair, ckey, N, i, i - 1);
  const int64_t dir = dn > dp ? 1 : -1;
  const int dmin = dir > 0 ? dp : dn;
  int64_t lmax = 2;
  while (delta_pk(cpair, ckey, N, i, i + lmax * dir) > dmin) lmax <<= 1;
  int64_t l = 0;
  for (int64_t t = lmax >> 1; t >= 1; t >>= 1)
    if (delta_pk(cpair, ckey, N, i, i + (l + t) * dir) > dmin) l += t;
  const int64_t j = i + l * dir;
  const int dnode = delta_pk(cpair, ckey, N, i, j);
  int64_t s = 0, t = l;
  do {
    t = (t + 1) >> 1;
    if (delta_pk(cpair, ckey, N, i, i + (s + t) * dir) > dnode) s += t;
  } while (t > 1);
  const int64_t gamma = i + s * dir + (dir < 0 ? -1 : 0);
  const int64_t lo = i < j ? i : j, hi = i < j ? j : i;
  const int32_t left = (lo == gamma) ? (int32_t)~gamma : (int32_t)gamma;
  const int32_t right = (hi == gamma + 1) ? (int32_t)~(gamma + 1) : (int32_t)(gamma + 1);
  iaux[i] = make_int4(left, right, (int)lo, (int)hi);
  if (left >= 0) iparent[gamma] = (int32_t)i;
  if (right >= 0) iparent[gamma + 1] = (int32_t)i;
  if (i == 0) iparent[0] = -1;
}

// Depth of every internal node (the root has depth 0), by climbing the
// parent links; read-only, so no thread waits for another.  maxd receives
// the largest depth.
__global__ void k_node_depth(const int32_t* __restrict__ iparent, int64_t N, int32_t* __restrict__ depth,
                             int32_t* __restrict__ maxd) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int d = 0;
  if (g < N - 1) {
    for (int32_t p = iparent[g]; p >= 0 && d < N; p = iparent[p]) ++d;  // d < N: stop on a malformed chain
    depth[g] = d;
  }
  for (int o = WAVE / 2; o > 0; o >>= 1) d = max(d, __shfl_xor(d, o));
  d = block_total(d, [](int a, int b) { return a > b ? a : b; });  // every lane holds its wave's max
  if (threadIdx.x == 0) atomicMax(maxd, d);
}

// Bottom-up tight boxes and heights, one depth level per launch: the nodes
// at depth d combine their children (cells, or nodes of depth d + 1 that the
// previous launch computed).  Launch boundaries order the levels, so no
// fences or counters are needed.
__global__ void k_level_boxes(const int2* __restrict__ cij, int64_t N, const int4* __restrict__ iaux,
                              const int32_t* __restrict__ depth, int d, int4* __restrict__ ibox,
                              int32_t* __restrict__ iheight) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N - 1 || depth[g] != d) return;
  const int4 a = iaux[g];
  int4 bx[2];
  int hh[2];
  const int32_t ch[2] = {a.x, a.y};
  for (int q = 0; q < 2; ++q) {
    if (ch[q] < 0) {
      const int2 v = cij[~ch[q]];
      bx[q] = make_int4(v.x, v.y, v.x, v.y);
      hh[q] = 0;
    } else {
      bx[q] = ibox[ch[q]];
      hh[q] = iheight[ch[q]];
    }
  }
  ibox[g] = make_int4(min(bx[0].x, bx[1].x), min(bx[0].y, bx[1].y), max(bx[0].z, bx[1].z), max(bx[0].w, bx[1].w));
  iheight[g] = 1 + max(hh[0], hh[1]);
}

inline unsigned blocks(int64_t n, int bs = 256) { return (unsigned)(n > 0 ? ceil_div(n, bs) : 1); }

}  // namespace

// ================================================================ launchers ==
#define LAUNCH(kern, n, ...) \
  do { if ((n) > 0) hipLaunchKernelGGL(kern, dim3(blocks(n)), dim3(256), 0, st, __VA_ARGS__); } while (0)

void launch_load(const SegDesc* segs, int nseg, int64_t total, int dtype, double* pb, double* pd, uint32_t* psd,
                 uint64_t* kw0, uint64_t* kw1, uint64_t* kw2, int32_t* perr, hipStream_t st) {
  LAUNCH(k_load, total, segs, nseg, total, dtype, pb, pd, psd, kw0, kw1, kw2, perr);
}
void launch_group_heads(const uint32_t* perm, const uint64_t* kw2s, const double* pb, const double* pd, int64_t n,
                        uint32_t* head, hipStream_t st) {
  LAUNCH(k_group_heads, n, perm, kw2s, pb, pd, n, head);
}
void launch_group_fill(const uint32_t* perm, const uint64_t* kw2s, const uint32_t* head, const uint32_t* gidx,
                       const double* pb, const double* pd, const uint32_t* psd, int64_t n, double* gb, double* gd,
                       uint32_t* gpair, int32_t* gw, hipStream_t st) {
  LAUNCH(k_group_fill, n, perm, kw2s, head, gidx, pb, pd, psd, n, gb, gd, gpair, gw);
}
void launch_count_total64(const uint64_t* cnt, const uint64_t* scanned, int64_t n, uint64_t* out, hipStream_t st) {
  hipLaunchKernelGGL(k_count_total64, dim3(1), dim3(64), 0, st, cnt, scanned, n, out);
}
void launch_count_total(const uint32_t* head, const uint32_t* scanned, int64_t n, uint64_t* out, hipStream_t st) {
  hipLaunchKernelGGL(k_count_total, dim3(1), dim3(64), 0, st, head, scanned, n, out);
}
void launch_nonzero_flags(const int32_t* gw, int64_t G, uint32_t* flag, hipStream_t st) {
  LAUNCH(k_nonzero_flags, G, gw, G, flag);
}
void launch_loc_fill(const int32_t* gw, const uint32_t* flag, const uint32_t* lidx, const double* gb, const double* gd,
                     const uint32_t* gpair, int64_t G, double* lb, double* ld, int32_t* lw, uint32_t* lpair,
                     const PairArrays& P, hipStream_t st) {
  LAUNCH(k_loc_fill, G, gw, flag, lidx, gb, gd, gpair, G, lb, ld, lw, lpair, P);
}
void launch_loc_bbox(const double* lb, const double* ld, const uint32_t* lpair, int64_t M, const PairArrays& P,
                     hipStream_t st) {
  LAUNCH(k_loc_bbox, M, lb, ld, lpair, M, P);
}
void launch_bucket_setup(const PairArrays& P, int64_t K, int64_t* nbuckets, hipStream_t st) {
  LAUNCH(k_bucket_setup, K, P, K, nbuckets);
}
void launch_bucket_count(const double* lb, const double* ld, const int32_t* lw, const uint32_t* lpair, int64_t M,
                         const PairArrays& P, uint32_t* bincnt, int64_t* lbin, hipStream_t st) {
  LAUNCH(k_bucket_count, M, lb, ld, lw, lpair, M, P, bincnt, lbin);
}
void launch_bucket_fill(const double* lb, const double* ld, const int64_t* lbin, int64_t M, const uint32_t* binstart,
                        uint32_t* bincur, double2* ent, uint32_t* entl, hipStream_t st) {
  LAUNCH(k_bucket_fill, M, lb, ld, lbin, M, binstart, bincur, ent, entl);
}
void launch_nn(const double* lb, const double* ld, const int32_t* lw, const uint32_t* lpair, int64_t M,
               const PairArrays& P, const uint32_t* binstart, const double2* ent, const uint32_t* entl, int64_t nbins,
               double* lt, double* lterm, bool l2, hipStream_t st) {
  if (l2) {
    LAUNCH(k_nn_init<true>, M, lb, ld, lw, M, lt, lterm);
  } else {
    LAUNCH(k_nn_init<false>, M, lb, ld, lw, M, lt, lterm);
  }
  if (nbins > 1)
    hipLaunchKernelGGL(l2 ? k_nn_bins<true> : k_nn_bins<false>, dim3((unsigned)(nbins - 1)), dim3(WAVE), 0, st, lw,
                       lpair, P, binstart, ent, entl, lt, lterm);
}
void launch_term_max(const double* lterm, const int32_t* lw, const uint32_t* lpair, int64_t M, const PairArrays& P,
                     hipStream_t st) {
  LAUNCH(k_term_max, M, lterm, lw, lpair, M, P);
}
void launch_rwmd_shift(const PairArrays& P, int64_t K, hipStream_t st) { LAUNCH(k_rwmd_shift, K, P, K); }
void launch_term_sum(const double* lterm, const int32_t* lw, const uint32_t* lpair, int64_t M, const PairArrays& P,
                     hipStream_t st) {
  LAUNCH(k_term_sum, M, lterm, lw, lpair, M, P);
}
void launch_params(const PairArrays& P, int64_t K, double eps_c, bool l2, hipStream_t st) {
  LAUNCH(k_params, K, P, K, eps_c, l2 ? 1 : 0);
}
void launch_snap(const double* lb, const double* ld, const uint32_t* lpair, int64_t M, const PairArrays& P, int64_t* li,
                 int64_t* lj, hipStream_t st) {
  LAUNCH(k_snap, M, lb, ld, lpair, M, P, li, lj);
}
void launch_morton(const int64_t* li, const int64_t* lj, const uint32_t* lpair, int64_t M, const PairArrays& P,
                   uint64_t* kw0, uint64_t* kw1, hipStream_t st) {
  LAUNCH(k_morton, M, li, lj, lpair, M, P, kw0, kw1);
}
void launch_cell_heads(const uint32_t* perm, const uint64_t* kw1s, const uint64_t* kw0, int64_t M, uint32_t* head,
                       hipStream_t st) {
  LAUNCH(k_cell_heads, M, perm, kw1s, kw0, M, head);
}
void launch_cell_fill(const uint32_t* perm, const uint64_t* kw1s, const uint64_t* kw0, const uint32_t* head,
                      const uint32_t* cidx, const int64_t* li, const int64_t* lj, const int32_t* lw, int64_t M,
                      const PairArrays& P, uint64_t* ckey, uint32_t* cpair, int2* cij, int32_t* ca, int32_t* cb,
                      hipStream_t st) {
  LAUNCH(k_cell_fill, M, perm, kw1s, kw0, head, cidx, li, lj, lw, M, P, ckey, cpair, cij, ca, cb);
}
void launch_run_bounds(const uint32_t* key, int64_t n, int64_t* lo, int64_t* hi, hipStream_t st) {
  LAUNCH(k_run_bounds, n, key, n, lo, hi);
}
void launch_bounds_count32(const int64_t* lo, const int64_t* hi, int64_t K, int32_t* out, hipStream_t st) {
  LAUNCH(k_bounds_count32, K, lo, hi, K, out);
}
void launch_karras(const uint32_t* cpair, const uint64_t* ckey, int64_t N, int4* iaux, int32_t* iparent,
                   hipStream_t st) {
  LAUNCH(k_karras, N - 1, cpair, ckey, N, iaux, iparent);
}
void launch_node_depth(const int32_t* iparent, int64_t N, int32_t* depth, int32_t* maxd, hipStream_t st) {
  if (N >= 2) LAUNCH(k_node_depth, N - 1, iparent, N, depth, maxd);
}
void launch_level_boxes(const int2* cij, int64_t N, const int4* iaux, const int32_t* depth, int d, int4* ibox,
                        int32_t* iheight, hipStream_t st) {
  if (N >= 2) LAUNCH(k_level_boxes, N - 1, cij, N, iaux, depth, d, ibox, iheight);
}
}  // namespace w1
