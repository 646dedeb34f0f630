// Learned surrogate for nearest-neighbour search over persistence diagrams:
// a DeepSets network
//   h1 = ReLU(W1 x + b1),  x = (birth, death - birth)      (2 -> 128)
//   h2 = ReLU(W2 h1 + b2)                                   (128 -> 128)
//   pool = sum of h2 over the points of the diagram
//   e = W3 pool + b3                                        (128 -> 64)
// with predicted distance ||e_A - e_B||_2.
//
// Precision: W1, b1 and W2 act in BF16, x enters as a two-term BF16
// expansion (hi + lo, about 16 significant bits), h1 is rounded to BF16;
// products accumulate in FP32 on the matrix cores; b2, pooling, rho and the
// optimizer are FP32, the loss FP64.  Master parameters are FP32.
//
// Both layers of phi run on MFMA (v_mfma_f32_16x16x32_bf16).  Layer 1 treats
// x as a K = 32 operand with five live slots (b_hi, b_lo, p_hi, p_lo, 1).
// The K order of layer 2 is permuted so that the accumulator layout of
// layer 1 is already the operand layout of layer 2: no LDS round trip.
// Every reduction has a fixed order, so results repeat bit for bit.
#include <type_traits>

#include "../../include/w1approx.h"
#include "surrogate.h"

namespace w1 {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

// FP32 -> BF16 bits, round to nearest, ties to even (finite inputs).
__device__ inline uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
// Hardware FP32 -> BF16 conversion (v_cvt_pk_bf16_f32, round to nearest even,
// the same rounding as f2bf for finite values).
__device__ inline __bf16 to_bf16(float f) { return (__bf16)f; }
// ReLU as an integer max on the bit pattern: negative floats (sign bit set)
// are negative integers, so max(bits, 0) maps them (and -0) to +0 and keeps
// positive values; one instruction, no NaN canonicalisation.
__device__ inline float relu(float v) { return __int_as_float(max(__float_as_int(v), 0)); }

__device__ inline bf16x8 as_bf16x8(u16x8 v) { return __builtin_bit_cast(bf16x8, v); }

__device__ inline f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

inline unsigned nblk(int64_t n, int b = 256) { return (unsigned)(n > 0 ? ceil_div(n, b) : 1); }

// Segment holding packed element p: the last one with out_off <= p (empty
// segments share their successor's offset and are never selected).
__device__ inline int find_seg(const SegDesc* segs, int nseg, int64_t p) {
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (segs[mid].out_off <= p) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__device__ inline void load_point(const SegDesc& sg, int64_t k, int dtype, double& b, double& d) {
  if (dtype == W1_F32) {
    b = ((const float*)sg.ptr)[2 * k];
    d = ((const float*)sg.ptr)[2 * k + 1];
  } else {
    b = ((const double*)sg.ptr)[2 * k];
    d = ((const double*)sg.ptr)[2 * k + 1];
  }
}

// ------------------------------------------------------------ packing --
// flag[p] = 1 for off-diagonal points, 0 for diagonal ones; invalid rows
// (non-finite, death < birth) set *err.  flag[total] = 0 (scan sentinel).
__global__ void k_ds_flags(const SegDesc* __restrict__ segs, int nseg, int64_t total, int dtype,
                           uint32_t* __restrict__ flag, int32_t* __restrict__ err) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p > total) return;
  if (p == total) {
    flag[p] = 0;
    return;
  }
  const SegDesc sg = segs[find_seg(segs, nseg, p)];
  double b, d;
  load_point(sg, p - sg.out_off, dtype, b, d);
  uint32_t f = 0;
  if (!(isfinite(b) && isfinite(d)) || d < b) atomicOr(err, 1);
  else f = d > b ? 1u : 0u;
  flag[p] = f;
}

__global__ void k_ds_scatter(const SegDesc* __restrict__ segs, int nseg, int64_t total, int dtype,
                             const uint32_t* __restrict__ flag, const uint32_t* __restrict__ pos,
                             float2* __restrict__ X) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= total || !flag[p]) return;
  const SegDesc sg = segs[find_seg(segs, nseg, p)];
  double b, d;
  load_point(sg, p - sg.out_off, dtype, b, d);
  X[pos[p]] = make_float2((float)b, (float)(d - b));
}

__global__ void k_ds_seg_starts(const SegDesc* __restrict__ segs, int nseg, const uint32_t* __restrict__ pos,
                                int64_t total, int64_t* __restrict__ dstart) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > nseg) return;
  dstart[i] = i < nseg ? (int64_t)pos[segs[i].out_off] : (int64_t)pos[total];
}

// ----------------------------------------------------------- operands --
// Lane l of a 16x16x32 MFMA supplies row (l % 16) of A / column (l % 16) of
// B and holds accumulator rows 4 (l / 16) .. +3 of column (l % 16).  Slot
// (g = l / 16, e) of A meets slot (g, e) of B.
//
// Layer 1, k-block kb: A row k = 16 kb + (l % 16); slots of lane group 0 are
// (w0, w0, w1, w1, b1, 0, 0, 0), all other slots 0.
// Layer 2, n-block nb, k-step ks: A row n = 16 nb + (l % 16); slot (g, e)
// holds K index 32 ks + 4 g + e (e < 4) or 32 ks + 16 + 4 g + (e - 4)
// (e >= 4): the rows that lane group g of the layer-1 accumulators holds.
__device__ inline int l2_k(int ks, int g, int e) { return e < 4 ? 32 * ks + 4 * g + e : 32 * ks + 16 + 4 * g + e - 4; }

__global__ void k_ds_prep(const float* __restrict__ P, uint16_t* __restrict__ w1op, uint16_t* __restrict__ w2op,
                          uint16_t* __restrict__ w2t) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;  // 0 .. 16383
  if (i < 8 * 64) {
    const int kb = i >> 6, lane = i & 63, r = lane & 15, g = lane >> 4;
    const int k = 16 * kb + r;
    uint16_t v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (g == 0) {
      const uint16_t w0 = f2bf(P[DS_OFF_W1 + 2 * k]), w1 = f2bf(P[DS_OFF_W1 + 2 * k + 1]);
      v[0] = w0;
      v[1] = w0;
      v[2] = w1;
      v[3] = w1;
      v[4] = f2bf(P[DS_OFF_B1 + k]);
    }
    for (int e = 0; e < 8; ++e) w1op[i * 8 + e] = v[e];
  }
  if (i < 8 * 4 * 64) {
    const int nb = i >> 8, ks = (i >> 6) & 3, lane = i & 63, r = lane & 15, g = lane >> 4;
    const int n = 16 * nb + r;
    for (int e = 0; e < 8; ++e) w2op[i * 8 + e] = f2bf(P[DS_OFF_W2 + n * DS_H + l2_k(ks, g, e)]);
  }
  {
    const int k = i >> 7, n = i & 127;
    w2t[i] = f2bf(P[DS_OFF_W2 + n * DS_H + k]);
  }
}

// -------------------------------------------------------- forward pass --
// One block (4 waves) per diagram; wave w takes 16-point tiles w, w + 4, ...
// Lane (r = l % 16, g = l / 16) handles point r of the tile and, after
// layer 2, the 32 units n = 16 nb + 4 g + q.
template <bool TRAIN>
__device__ __forceinline__ void embed_body(const float2* __restrict__ X, const int64_t* __restrict__ dstart,
                                           const int32_t* __restrict__ dlist, const float* __restrict__ P,
                                           const u16x8* __restrict__ w1op, const u16x8* __restrict__ w2op,
                                           float* __restrict__ pool_out, float* __restrict__ emb_out,
                                           const DsTrainRows& tr) {
  __shared__ bf16x8 s_w1[8 * 64];      // layer-1 operands (4 KiB)
  __shared__ f32x4 s_b2[8 * 4];        // b2 in accumulator layout: [nb][g] -> units 16 nb + 4 g + q
  __shared__ float s_part[4][DS_H];
  __shared__ float s_pool[DS_H];
  __shared__ int32_t s_cnt[4][DS_H];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = lane & 15, g = lane >> 4;
  const int64_t d = blockIdx.x;
  const int64_t src = dlist ? dlist[d] : d;
  const int64_t oi = TRAIN ? d : src;  // output row: batch slot, or the diagram itself
  const int64_t start = dstart[src];
  const int64_t n = dstart[src + 1] - start;
  const int64_t nrows = TRAIN ? ((n + 31) & ~int64_t(31)) : n;
  const int64_t ntiles = (nrows + 15) >> 4;

  for (int i = threadIdx.x; i < 8 * 64; i += 256) s_w1[i] = as_bf16x8(w1op[i]);
  bf16x8 a2[8][4];  // layer-2 operands stay in registers for the whole diagram
  for (int nb = 0; nb < 8; ++nb)
    for (int ks = 0; ks < 4; ++ks) a2[nb][ks] = as_bf16x8(w2op[(nb * 4 + ks) * 64 + lane]);
  if (threadIdx.x < 32) {
    const int nb = threadIdx.x >> 2, gg = threadIdx.x & 3;
    for (int q = 0; q < 4; ++q) s_b2[threadIdx.x][q] = P[DS_OFF_B2 + 16 * nb + 4 * gg + q];
  }
  f32x4 acc_pool[8];
  int cnt[8][4];
  for (int nb = 0; nb < 8; ++nb)
    for (int q = 0; q < 4; ++q) {
      acc_pool[nb][q] = 0.f;
      cnt[nb][q] = 0;
    }
  __syncthreads();

  // the next tile's point is loaded one iteration ahead (hides its latency)
  float2 x_next = make_float2(0.f, 0.f);
  if (wave * 16 + r < n) x_next = X[start + wave * 16 + r];
  // One 16-point tile.  MASKED handles a tile that may hold points past the
  // end (only a diagram's last tile, or any tile when training, which also
  // writes the padding rows); full tiles take the path without per-lane
  // tests.
  auto tile = [&](int64_t t, auto masked_tag) {
    constexpr bool MASKED = decltype(masked_tag)::value;
    const int64_t p = t * 16 + r;
    const bool valid = !MASKED || p < n;
    const float2 x = x_next;
    const int64_t pn = p + 64;
    x_next = pn < n ? X[start + pn] : make_float2(0.f, 0.f);
    const __bf16 bh = to_bf16(x.x), ph = to_bf16(x.y);
    const __bf16 bl = to_bf16(x.x - (float)bh), pl = to_bf16(x.y - (float)ph);
    const __bf16 z0 = (__bf16)0.f, one = (__bf16)1.f;
    bf16x8 b1 = {z0, z0, z0, z0, z0, z0, z0, z0};
    if (g == 0 && valid) b1 = bf16x8{bh, bl, ph, pl, one, z0, z0, z0};

    // layer 1: h1[k][r] for k = 16 kb + 4 g + q
    bf16x8 hb[4];
    for (int kb = 0; kb < 8; ++kb) {
      if (kb == 4) __builtin_amdgcn_sched_barrier(0);  // two halves: 16 live accumulators
      const f32x4 z = mfma(s_w1[kb * 64 + lane], b1, f32x4{0.f, 0.f, 0.f, 0.f});
      for (int q = 0; q < 4; ++q) hb[kb >> 1][(kb & 1) * 4 + q] = to_bf16(relu(z[q]));
    }
    __builtin_amdgcn_sched_barrier(0);
    // layer 2: z2[n][r] for n = 16 nb + 4 g + q, pooled two output blocks at
    // a time (their MFMA chains interleave; few accumulators are live)
    uint32_t bits = 0;
    for (int nb = 0; nb < 8; nb += 2) {
      f32x4 c0 = s_b2[nb * 4 + g], c1 = s_b2[(nb + 1) * 4 + g];
      for (int ks = 0; ks < 4; ++ks) {
        c0 = mfma(a2[nb][ks], hb[ks], c0);
        c1 = mfma(a2[nb + 1][ks], hb[ks], c1);
      }
      for (int q = 0; q < 4; ++q) {
        if constexpr (MASKED) {
          acc_pool[nb][q] += valid ? relu(c0[q]) : 0.f;
          acc_pool[nb + 1][q] += valid ? relu(c1[q]) : 0.f;
        } else {
          acc_pool[nb][q] += relu(c0[q]);
          acc_pool[nb + 1][q] += relu(c1[q]);
        }
      }
      if constexpr (TRAIN)
        for (int q = 0; q < 4; ++q) {
          const bool on0 = valid && c0[q] > 0.f, on1 = valid && c1[q] > 0.f;
          bits |= ((on0 ? 1u : 0u) << (nb * 4 + q)) | ((on1 ? 1u : 0u) << ((nb + 1) * 4 + q));
          cnt[nb][q] += on0 ? 1 : 0;
          cnt[nb + 1][q] += on1 ? 1 : 0;
        }
    }
    if constexpr (TRAIN) {
      const int64_t row = tr.roff[d] + p;
      tr.m2[row * 4 + g] = bits;
      for (int kb = 0; kb < 8; ++kb) {
        const int k0 = 16 * kb + 4 * g;
        const int base = (kb & 1) * 4;
        const u16x8 hv = __builtin_bit_cast(u16x8, hb[kb >> 1]);
        uint2 pk;
        pk.x = (uint32_t)hv[base] | ((uint32_t)hv[base + 1] << 16);
        pk.y = (uint32_t)hv[base + 2] | ((uint32_t)hv[base + 3] << 16);
        *(uint2*)(tr.h1 + row * DS_H + k0) = pk;
        for (int q = 0; q < 4; ++q) tr.h1t[(int64_t)(k0 + q) * tr.rows + row] = hv[base + q];
      }
      if (g == 0) tr.xb[row] = make_float2((float)bh + (float)bl, (float)ph + (float)pl);
    }
  };
  for (int64_t t = wave; t < ntiles; t += 4) {
    if (!TRAIN && t * 16 + 16 <= n) tile(t, std::false_type{});
    else tile(t, std::true_type{});
  }

  // pool: sum over the 16 points of each lane group (butterfly: every lane
  // ends with the same bits), then over the 4 waves in order.
  for (int nb = 0; nb < 8; ++nb)
    for (int q = 0; q < 4; ++q) {
      float v = acc_pool[nb][q];
      for (int o = 1; o < 16; o <<= 1) v += __shfl_xor(v, o);
      acc_pool[nb][q] = v;
      if constexpr (TRAIN) {
        int c = cnt[nb][q];
        for (int o = 1; o < 16; o <<= 1) c += __shfl_xor(c, o);
        cnt[nb][q] = c;
      }
    }
  if (r == 0) {
    for (int nb = 0; nb < 8; ++nb)
      for (int q = 0; q < 4; ++q) {
        s_part[wave][16 * nb + 4 * g + q] = acc_pool[nb][q];
        if constexpr (TRAIN) s_cnt[wave][16 * nb + 4 * g + q] = cnt[nb][q];
      }
  }
  __syncthreads();
  if (threadIdx.x < DS_H) {
    const int u = threadIdx.x;
    const float v = ((s_part[0][u] + s_part[1][u]) + s_part[2][u]) + s_part[3][u];
    s_pool[u] = v;
    pool_out[oi * DS_H + u] = v;
    if constexpr (TRAIN) tr.cnt2[d * DS_H + u] = s_cnt[0][u] + s_cnt[1][u] + s_cnt[2][u] + s_cnt[3][u];
  }
  __syncthreads();
  // rho: output o = t / 4, quarter t % 4 of the 128 inputs
  {
    const int o = threadIdx.x >> 2, part = threadIdx.x & 3;
    float s = 0.f;
    for (int u = 32 * part; u < 32 * part + 32; ++u) s = fmaf(P[DS_OFF_W3 + o * DS_H + u], s_pool[u], s);
    s += __shfl_xor(s, 1);
    s += __shfl_xor(s, 2);
    if (part == 0) emb_out[oi * DS_E + o] = s + P[DS_OFF_B3 + o];
  }
}

// Inference: two blocks (eight waves) per CU, the layer-2 operands resident
// in registers.
__global__ void __launch_bounds__(256, 2) k_ds_embed_fwd(const float2* __restrict__ X,
                                                         const int64_t* __restrict__ dstart,
                                                         const int32_t* __restrict__ dlist, const float* __restrict__ P,
                                                         const u16x8* __restrict__ w1op, const u16x8* __restrict__ w2op,
                                                         float* __restrict__ pool_out, float* __restrict__ emb_out) {
  embed_body<false>(X, dstart, dlist, P, w1op, w2op, pool_out, emb_out, DsTrainRows{});
}

// Training forward: also writes the per-row tensors the backward pass reads.
__global__ void __launch_bounds__(256) k_ds_embed_train(const float2* __restrict__ X, const int64_t* __restrict__ dstart,
                                                        const int32_t* __restrict__ dlist, const float* __restrict__ P,
                                                        const u16x8* __restrict__ w1op, const u16x8* __restrict__ w2op,
                                                        float* __restrict__ pool_out, float* __restrict__ emb_out,
                                                        DsTrainRows tr) {
  embed_body<true>(X, dstart, dlist, P, w1op, w2op, pool_out, emb_out, tr);
}

// ------------------------------------------------------------ backward --
// Relative squared error of each pair: ((||e_a - e_b|| - w) / w)^2 / P;
// gp = d loss / d e_a (= -d loss / d e_b).
__global__ void k_ds_loss(const float* __restrict__ emb, const int32_t* __restrict__ pa,
                          const int32_t* __restrict__ pb, const double* __restrict__ w, int64_t P,
                          float* __restrict__ gp, double* __restrict__ lpart) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P) return;
  const float* ea = emb + (int64_t)pa[i] * DS_E;
  const float* eb = emb + (int64_t)pb[i] * DS_E;
  double s = 0.0;
  for (int o = 0; o < DS_E; ++o) {
    const double t = (double)ea[o] - (double)eb[o];
    s += t * t;
  }
  const double pred = sqrt(s);
  const double rel = (pred - w[i]) / w[i];
  lpart[i] = rel * rel / (double)P;
  const double f = pred > 0.0 ? 2.0 * rel / (w[i] * (double)P) / pred : 0.0;
  for (int o = 0; o < DS_E; ++o) gp[i * DS_E + o] = (float)(f * ((double)ea[o] - (double)eb[o]));
}

// demb[d] = sum over the pairs of diagram d, in list order, of +gp (as the
// first diagram) or -gp (as the second).  occ entry = 2 * pair + side.
__global__ void k_ds_demb(const float* __restrict__ gp, const int32_t* __restrict__ occ_start,
                          const int32_t* __restrict__ occ, float* __restrict__ demb) {
  const int64_t d = blockIdx.x;
  const int o = threadIdx.x;
  float s = 0.f;
  for (int j = occ_start[d]; j < occ_start[d + 1]; ++j) {
    const int32_t e = occ[j];
    const float v = gp[(int64_t)(e >> 1) * DS_E + o];
    s += (e & 1) ? -v : v;
  }
  demb[d * DS_E + o] = s;
}

__global__ void k_ds_dW3(const float* __restrict__ demb, const float* __restrict__ pool, int64_t D,
                         float* __restrict__ grad) {
  const int o = blockIdx.x, u = threadIdx.x;
  float s = 0.f, sb = 0.f;
  for (int64_t d = 0; d < D; ++d) {
    const float g = demb[d * DS_E + o];
    s = fmaf(g, pool[d * DS_H + u], s);
    sb += g;
  }
  grad[DS_OFF_W3 + o * DS_H + u] = s;
  if (u == 0) grad[DS_OFF_B3 + o] = sb;
}

__global__ void k_ds_dpool(const float* __restrict__ demb, const float* __restrict__ P, float* __restrict__ dpool) {
  const int64_t d = blockIdx.x;
  const int u = threadIdx.x;
  float s = 0.f;
  for (int o = 0; o < DS_E; ++o) s = fmaf(P[DS_OFF_W3 + o * DS_H + u], demb[d * DS_E + o], s);
  dpool[d * DS_H + u] = s;
}

// db2[u] = sum_d dpool[d][u] * (rows of d with unit u active).
__global__ void k_ds_db2(const float* __restrict__ dpool, const int32_t* __restrict__ cnt2, int64_t D,
                         float* __restrict__ grad) {
  const int u = threadIdx.x;
  float s = 0.f;
  for (int64_t d = 0; d < D; ++d) s = fmaf(dpool[d * DS_H + u], (float)cnt2[d * DS_H + u], s);
  grad[DS_OFF_B2 + u] = s;
}

// dZ2[row][u] = bf16(dpool[diagram of row][u]) if unit u was active, else 0;
// written row-major and transposed (32-row tiles through LDS).
__global__ void __launch_bounds__(256) k_ds_dz2(const uint32_t* __restrict__ m2, const float* __restrict__ dpool,
                                                const int64_t* __restrict__ roff, int64_t D, int64_t rows,
                                                uint16_t* __restrict__ dz2, uint16_t* __restrict__ dz2t) {
  __shared__ uint16_t tile[32][DS_H + 2];
  const int64_t row0 = (int64_t)blockIdx.x * 32;
  for (int i = threadIdx.x; i < 32 * DS_H; i += 256) {
    const int rr = i >> 7, u = i & 127;
    const int64_t row = row0 + rr;
    int lo = 0, hi = (int)D - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (roff[mid] <= row) lo = mid;
      else hi = mid - 1;
    }
    const int g = (u >> 2) & 3, bit = (u >> 4) * 4 + (u & 3);
    const bool on = (m2[row * 4 + g] >> bit) & 1u;
    const uint16_t v = on ? f2bf(dpool[(int64_t)lo * DS_H + u]) : (uint16_t)0;
    dz2[row * DS_H + u] = v;
    tile[rr][u] = v;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 32 * DS_H; i += 256) {
    const int u = i >> 5, rr = i & 31;
    dz2t[(int64_t)u * rows + row0 + rr] = tile[rr][u];
  }
}

// Partial sums over row slice z: dW1[k][0..1] and db1[k] from dZ1 = dH1 where
// h1 > 0.  part[z] = (dW1 as [k][2], db1).
__global__ void k_ds_dlayer1(const float* __restrict__ dh1, const uint16_t* __restrict__ h1,
                             const float2* __restrict__ xb, int64_t rows, int64_t slice, float* __restrict__ part) {
  const int64_t z = blockIdx.x;
  const int k = threadIdx.x;
  float g0 = 0.f, g1 = 0.f, gb = 0.f;
  const int64_t end = min(rows, (z + 1) * slice);
  for (int64_t p = z * slice; p < end; ++p) {
    if (h1[p * DS_H + k] == 0) continue;  // ReLU inactive, or a padding row
    const float g = dh1[p * DS_H + k];
    const float2 x = xb[p];
    g0 = fmaf(g, x.x, g0);
    g1 = fmaf(g, x.y, g1);
    gb += g;
  }
  part[z * 384 + 2 * k] = g0;
  part[z * 384 + 2 * k + 1] = g1;
  part[z * 384 + 256 + k] = gb;
}

// C[z] (M x N, FP32, row-major) = A[:, kz] Bt[:, kz]^T over K slice z.  A is
// M x K and Bt is N x K, BF16 row-major.  M, N, K, kslice multiples of 32.
// One wave per 32 x 32 output tile, four MFMAs per K step of 32.
__global__ void __launch_bounds__(64) k_gemm_nt(const uint16_t* __restrict__ A, const uint16_t* __restrict__ Bt,
                                                float* __restrict__ C, int64_t M, int64_t N, int64_t K,
                                                int64_t kslice) {
  const int lane = threadIdx.x;
  const int64_t m0 = (int64_t)blockIdx.x * 32, n0 = (int64_t)blockIdx.y * 32;
  const int64_t z = blockIdx.z;
  const int64_t k0 = z * kslice, k1 = min(K, k0 + kslice);
  const int r = lane & 15, g = lane >> 4;
  f32x4 acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int64_t k = k0; k < k1; k += 32) {
    bf16x8 a[2], b[2];
    for (int i = 0; i < 2; ++i) a[i] = as_bf16x8(*(const u16x8*)(A + (m0 + 16 * i + r) * K + k + 8 * g));
    for (int j = 0; j < 2; ++j) b[j] = as_bf16x8(*(const u16x8*)(Bt + (n0 + 16 * j + r) * K + k + 8 * g));
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j) acc[i][j] = mfma(a[i], b[j], acc[i][j]);
  }
  float* Cz = C + z * M * N;
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      for (int q = 0; q < 4; ++q) Cz[(m0 + 16 * i + 4 * g + q) * N + n0 + 16 * j + r] = acc[i][j][q];
}

__global__ void k_sum_slices(const float* __restrict__ part, int64_t nz, int64_t n, float* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float s = 0.f;
  for (int64_t z = 0; z < nz; ++z) s += part[z * n + i];
  out[i] = s;
}

__global__ void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m1,
                       float* __restrict__ m2, int64_t n, float lr, float beta1, float beta2, float eps, float bc1,
                       float bc2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float a = beta1 * m1[i] + (1.f - beta1) * gi;
  const float b = beta2 * m2[i] + (1.f - beta2) * gi * gi;
  m1[i] = a;
  m2[i] = b;
  w[i] -= lr * (a / bc1) / (sqrtf(b / bc2) + eps);
}

// score[q][i] = ||embq[q] - embdb[i]||_2
__global__ void k_ds_scores(const float* __restrict__ eq, int64_t nq, const float* __restrict__ edb, int64_t m,
                            float* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t q = blockIdx.y;
  if (i >= m) return;
  float s = 0.f;
  for (int o = 0; o < DS_E; ++o) {
    const float t = eq[q * DS_E + o] - edb[i * DS_E + o];
    s = fmaf(t, t, s);
  }
  out[q * m + i] = sqrtf(s);
}

// Per-diagram sums of the dual-bound test functions, from the raw rows in
// FP64: S[d][0] = sum of h, S[d][j] = sum of max(0, h - 2^(j-21)) for
// j = 1..32, with h = (death - birth) / 2 the distance to the diagonal.
// Diagonal rows add 0; invalid rows (non-finite, death < birth) set *err.
// One block per diagram; per-thread partial sums over a stride of 256 rows,
// then a butterfly over each wave and the four waves in order.
__global__ void __launch_bounds__(256) k_nn_stats(const SegDesc* __restrict__ segs, int dtype,
                                                  double* __restrict__ S, int32_t* __restrict__ err) {
  __shared__ double s_w[4][NN_NSTATS];
  const SegDesc sg = segs[blockIdx.x];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double acc[NN_NSTATS];
  for (int j = 0; j < NN_NSTATS; ++j) acc[j] = 0.0;
  for (int64_t k = threadIdx.x; k < sg.n; k += 256) {
    double b, d;
    load_point(sg, k, dtype, b, d);
    if (!(isfinite(b) && isfinite(d)) || d < b) {
      atomicOr(err, 1);
      continue;
    }
    const double h = (d - b) * 0.5;
    acc[0] += h;
    for (int j = 1; j < NN_NSTATS; ++j) acc[j] += fmax(0.0, h - ldexp(1.0, j - 21));
  }
  for (int j = 0; j < NN_NSTATS; ++j) {
    double v = acc[j];
    for (int o = 1; o < 64; o <<= 1) v += __shfl_xor(v, o);
    if (lane == 0) s_w[wave][j] = v;
  }
  __syncthreads();
  if (threadIdx.x < NN_NSTATS) {
    const int j = threadIdx.x;
    S[(int64_t)blockIdx.x * NN_NSTATS + j] = ((s_w[0][j] + s_w[1][j]) + s_w[2][j]) + s_w[3][j];
  }
}

}  // namespace

void ds_flags(const SegDesc* segs, int nseg, int64_t total, int dtype, uint32_t* flag, int32_t* err, hipStream_t st) {
  hipLaunchKernelGGL(k_ds_flags, dim3(nblk(total + 1)), dim3(256), 0, st, segs, nseg, total, dtype, flag, err);
}
void ds_scatter(const SegDesc* segs, int nseg, int64_t total, int dtype, const uint32_t* flag, const uint32_t* pos,
                float2* X, hipStream_t st) {
  if (total <= 0) return;
  hipLaunchKernelGGL(k_ds_scatter, dim3(nblk(total)), dim3(256), 0, st, segs, nseg, total, dtype, flag, pos, X);
}
void ds_seg_starts(const SegDesc* segs, int nseg, const uint32_t* pos, int64_t total, int64_t* dstart,
                   hipStream_t st) {
  hipLaunchKernelGGL(k_ds_seg_starts, dim3(nblk(nseg + 1)), dim3(256), 0, st, segs, nseg, pos, total, dstart);
}
void ds_prep(const float* params, const DsOperands& op, hipStream_t st) {
  hipLaunchKernelGGL(k_ds_prep, dim3(64), dim3(256), 0, st, params, op.w1op, op.w2op, op.w2t);
}
void ds_embed(const float2* X, const int64_t* dstart, const int32_t* dlist, int64_t D, const float* params,
              const DsOperands& op, float* pool, float* emb, const DsTrainRows* train, hipStream_t st) {
  if (D <= 0) return;
  if (train)
    hipLaunchKernelGGL(k_ds_embed_train, dim3((unsigned)D), dim3(256), 0, st, X, dstart, dlist, params,
                       (const u16x8*)op.w1op, (const u16x8*)op.w2op, pool, emb, *train);
  else
    hipLaunchKernelGGL(k_ds_embed_fwd, dim3((unsigned)D), dim3(256), 0, st, X, dstart, dlist, params,
                       (const u16x8*)op.w1op, (const u16x8*)op.w2op, pool, emb);
}
void ds_loss(const float* emb, const int32_t* pa, const int32_t* pb, const double* w, int64_t P, float* gp,
             double* lpart, hipStream_t st) {
  hipLaunchKernelGGL(k_ds_loss, dim3(nblk(P, 64)), dim3(64), 0, st, emb, pa, pb, w, P, gp, lpart);
}
void ds_demb(const float* gp, const int32_t* occ_start, const int32_t* occ, int64_t D, float* demb, hipStream_t st) {
  hipLaunchKernelGGL(k_ds_demb, dim3((unsigned)D), dim3(DS_E), 0, st, gp, occ_start, occ, demb);
}
void ds_dW3(const float* demb, const float* pool, int64_t D, float* grad, hipStream_t st) {
  hipLaunchKernelGGL(k_ds_dW3, dim3(DS_E), dim3(DS_H), 0, st, demb, pool, D, grad);
}
void ds_dpool(const float* demb, const float* params, int64_t D, float* dpool, hipStream_t st) {
  hipLaunchKernelGGL(k_ds_dpool, dim3((unsigned)D), dim3(DS_H), 0, st, demb, params, dpool);
}
void ds_db2(const float* dpool, const int32_t* cnt2, int64_t D, float* grad, hipStream_t st) {
  hipLaunchKernelGGL(k_ds_db2, dim3(1), dim3(DS_H), 0, st, dpool, cnt2, D, grad);
}
void ds_dz2(const uint32_t* m2, const float* dpool, const int64_t* roff, int64_t D, int64_t rows, uint16_t* dz2,
            uint16_t* dz2t, hipStream_t st) {
  if (rows <= 0) return;
  hipLaunchKernelGGL(k_ds_dz2, dim3((unsigned)(rows / 32)), dim3(256), 0, st, m2, dpool, roff, D, rows, dz2, dz2t);
}
void ds_dlayer1(const float* dh1, const uint16_t* h1, const float2* xb, int64_t rows, int64_t slice, float* part,
                hipStream_t st) {
  hipLaunchKernelGGL(k_ds_dlayer1, dim3((unsigned)ceil_div(rows, slice)), dim3(DS_H), 0, st, dh1, h1, xb, rows,
                     slice, part);
}
void ds_gemm_nt(const uint16_t* A, const uint16_t* Bt, float* C, int64_t M, int64_t N, int64_t K, int64_t kslice,
                hipStream_t st) {
  const int64_t nz = ceil_div(K, kslice);
  hipLaunchKernelGGL(k_gemm_nt, dim3((unsigned)(M / 32), (unsigned)(N / 32), (unsigned)nz), dim3(64), 0, st, A, Bt, C,
                     M, N, K, kslice);
}
void ds_sum_slices(const float* part, int64_t nz, int64_t n, float* out, hipStream_t st) {
  hipLaunchKernelGGL(k_sum_slices, dim3(nblk(n)), dim3(256), 0, st, part, nz, n, out);
}
void ds_adam(float* w, const float* g, float* m1, float* m2, int64_t n, float lr, float beta1, float beta2, float eps,
             float bc1, float bc2, hipStream_t st) {
  hipLaunchKernelGGL(k_adam, dim3(nblk(n)), dim3(256), 0, st, w, g, m1, m2, n, lr, beta1, beta2, eps, bc1, bc2);
}
void nn_stats(const SegDesc* segs, int nseg, int dtype, double* S, int32_t* err, hipStream_t st) {
  if (nseg <= 0) return;
  hipLaunchKernelGGL(k_nn_stats, dim3((unsigned)nseg), dim3(256), 0, st, segs, dtype, S, err);
}
void ds_scores(const float* embq, int64_t nq, const float* embdb, int64_t m, float* out, hipStream_t st) {
  if (nq <= 0 || m <= 0) return;
  hipLaunchKernelGGL(k_ds_scores, dim3(nblk(m), (unsigned)nq), dim3(256), 0, st, embq, nq, embdb, m, out);
}

}  // namespace w1
