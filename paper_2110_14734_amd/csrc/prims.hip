// Device-wide primitives for the w1approx pipeline: exclusive scan
// (reduce-then-scan), stable LSD radix sort with wave-level multisplit
// ranking, fills and gathers.  All kernels use wave64 ballots and LDS; no
// vendor library is involved.
#include "common.h"

namespace w1 {

namespace {

constexpr int SB = 256;       // threads per block
constexpr int SI = 8;         // items per thread
constexpr int STILE = SB * SI;

template <typename T>
__device__ inline T wave_incl_scan(T v) {
  const int lane = lane_id();
#pragma unroll
  for (int d = 1; d < WAVE; d <<= 1) {
    T o = __shfl_up(v, d);
    if (lane >= d) v += o;
  }
  return v;
}

// Exclusive block scan of one value per thread; returns the prefix and the
// block total.
template <typename T>
__device__ inline T block_excl_scan(T v, T* s_wave, T* total) {
  const int lane = lane_id(), wave = threadIdx.x / WAVE;
  T inc = wave_incl_scan(v);
  if (lane == WAVE - 1) s_wave[wave] = inc;
  __syncthreads();
  T wpre = 0, tot = 0;
  for (int w = 0; w < SB / WAVE; ++w) {
    T x = s_wave[w];
    if (w < wave) wpre += x;
    tot += x;
  }
  __syncthreads();
  *total = tot;
  return wpre + inc - v;
}

template <typename T>
__global__ void __launch_bounds__(SB) k_scan_reduce(const T* __restrict__ in, T* __restrict__ part, int64_t n) {
  __shared__ T s_wave[SB / WAVE];
  const int64_t base = (int64_t)blockIdx.x * STILE;
  T acc = 0;
#pragma unroll
  for (int it = 0; it < SI; ++it) {
    int64_t x = base + (int64_t)it * SB + threadIdx.x;
    if (x < n) acc += in[x];
  }
  T tot;
  block_excl_scan(acc, s_wave, &tot);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

template <typename T>
__global__ void __launch_bounds__(SB) k_scan_down(const T* in, T* out, const T* __restrict__ part, int64_t n) {
  __shared__ T s_tile[STILE];
  __shared__ T s_wave[SB / WAVE];
  const int64_t base = (int64_t)blockIdx.x * STILE;
#pragma unroll
  for (int it = 0; it < SI; ++it) {
    int64_t x = base + (int64_t)it * SB + threadIdx.x;
    s_tile[it * SB + threadIdx.x] = x < n ? in[x] : T(0);
  }
  __syncthreads();
  T loc[SI];
  T run = 0;
#pragma unroll
  for (int k = 0; k < SI; ++k) {
    loc[k] = run;
    run += s_tile[threadIdx.x * SI + k];
  }
  T tot;
  T pre = block_excl_scan(run, s_wave, &tot);
  const T carry = part ? part[blockIdx.x] : T(0);
#pragma unroll
  for (int k = 0; k < SI; ++k) s_tile[threadIdx.x * SI + k] = carry + pre + loc[k];
  __syncthreads();
#pragma unroll
  for (int it = 0; it < SI; ++it) {
    int64_t x = base + (int64_t)it * SB + threadIdx.x;
    if (x < n) out[x] = s_tile[it * SB + threadIdx.x];
  }
}

template <typename T>
void scan_impl(const T* in, T* out, int64_t n, void* tmp, hipStream_t st) {
  if (n <= 0) return;
  int64_t nb = ceil_div(n, STILE);
  if (nb == 1) {
    hipLaunchKernelGGL(k_scan_down<T>, dim3(1), dim3(SB), 0, st, in, out, (const T*)nullptr, n);
    return;
  }
  T* part = (T*)tmp;
  void* rest = (void*)(part + ((nb + 63) / 64) * 64);
  hipLaunchKernelGGL(k_scan_reduce<T>, dim3((unsigned)nb), dim3(SB), 0, st, in, part, n);
  scan_impl<T>(part, part, nb, rest, st);
  hipLaunchKernelGGL(k_scan_down<T>, dim3((unsigned)nb), dim3(SB), 0, st, in, out, (const T*)part, n);
}

// ---------------------------------------------------------------- radix --
constexpr int RB = 256;       // threads per block
constexpr int RI = 8;         // keys per thread
constexpr int RTILE = RB * RI;

__global__ void __launch_bounds__(RB) k_radix_hist(const uint64_t* __restrict__ keys, int64_t n, int shift,
                                                  uint32_t* __restrict__ hist, int nb) {
  __shared__ uint32_t s_h[256];
  s_h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * RTILE;
#pragma unroll
  for (int it = 0; it < RI; ++it) {
    int64_t x = base + (int64_t)it * RB + threadIdx.x;
    if (x < n) atomicAdd(&s_h[(keys[x] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nb + blockIdx.x] = s_h[threadIdx.x];
}

__global__ void __launch_bounds__(RB) k_radix_scatter(const uint64_t* __restrict__ kin, const uint32_t* __restrict__ vin,
                                                     uint64_t* __restrict__ kout, uint32_t* __restrict__ vout,
                                                     int64_t n, int shift, const uint32_t* __restrict__ offs, int nb) {
  __shared__ uint32_t s_base[256];
  __shared__ uint32_t s_goff[256];
  __shared__ uint32_t s_wave[RB / WAVE][256];
  const int tid = threadIdx.x, wave = tid / WAVE;
  s_base[tid] = 0;
  s_goff[tid] = offs[(int64_t)tid * nb + blockIdx.x];
  const int64_t base = (int64_t)blockIdx.x * RTILE;
  const uint64_t below = lanes_below();
  for (int it = 0; it < RI; ++it) {
    for (int q = tid; q < (RB / WAVE) * 256; q += RB) (&s_wave[0][0])[q] = 0;
    const int64_t x = base + (int64_t)it * RB + tid;
    const bool valid = x < n;
    uint64_t key = valid ? kin[x] : 0;
    uint32_t val = valid ? vin[x] : 0;
    uint32_t digit = (uint32_t)(key >> shift) & 255u;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      uint64_t bal = __ballot((digit >> b) & 1u);
      peers &= ((digit >> b) & 1u) ? bal : ~bal;
    }
    const uint32_t rank = (uint32_t)__popcll(peers & below);
    __syncthreads();
    if (valid && rank == 0) s_wave[wave][digit] = (uint32_t)__popcll(peers);
    __syncthreads();
    {
      uint32_t run = s_base[tid];
#pragma unroll
      for (int w = 0; w < RB / WAVE; ++w) {
        uint32_t c = s_wave[w][tid];
        s_wave[w][tid] = run;
        run += c;
      }
      s_base[tid] = run;
    }
    __syncthreads();
    if (valid) {
      uint32_t pos = s_goff[digit] + s_wave[wave][digit] + rank;
      kout[pos] = key;
      vout[pos] = val;
    }
    __syncthreads();
  }
}

// OR and AND of all keys in two launches without atomics: per-block
// partials, then one block combines them.
__global__ void __launch_bounds__(256) k_or_and_part(const uint64_t* __restrict__ keys, int64_t n,
                                                     uint64_t* __restrict__ part) {
  __shared__ uint64_t s_o[4], s_a[4];
  uint64_t o = 0, a = ~0ull;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t k = keys[x];
    o |= k;
    a &= k;
  }
  for (int d = WAVE / 2; d > 0; d >>= 1) {
    o |= __shfl_xor(o, d);
    a &= __shfl_xor(a, d);
  }
  const int w = threadIdx.x / WAVE;
  if (lane_id() == 0) {
    s_o[w] = o;
    s_a[w] = a;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = s_o[0] | s_o[1] | s_o[2] | s_o[3];
    part[2 * blockIdx.x + 1] = s_a[0] & s_a[1] & s_a[2] & s_a[3];
  }
}

__global__ void __launch_bounds__(256) k_or_and_final(const uint64_t* __restrict__ part, int nparts,
                                                      uint64_t* __restrict__ out) {
  __shared__ uint64_t s_o[4], s_a[4];
  uint64_t o = 0, a = ~0ull;
  for (int b = threadIdx.x; b < nparts; b += blockDim.x) {
    o |= part[2 * b];
    a &= part[2 * b + 1];
  }
  for (int d = WAVE / 2; d > 0; d >>= 1) {
    o |= __shfl_xor(o, d);
    a &= __shfl_xor(a, d);
  }
  const int w = threadIdx.x / WAVE;
  if (lane_id() == 0) {
    s_o[w] = o;
    s_a[w] = a;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    out[0] = s_o[0] | s_o[1] | s_o[2] | s_o[3];
    out[1] = s_a[0] & s_a[1] & s_a[2] & s_a[3];
  }
}

template <typename T>
__global__ void k_fill(T* p, T v, int64_t n) {
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x) p[x] = v;
}

__global__ void k_iota(uint32_t* p, int64_t n) {
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x)
    p[x] = (uint32_t)x;
}

__global__ void k_gather64(const uint64_t* __restrict__ src, const uint32_t* __restrict__ idx, uint64_t* __restrict__ dst,
                           int64_t n) {
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x)
    dst[x] = src[idx[x]];
}

inline unsigned grid_for(int64_t n, int bs = 256) {
  int64_t g = ceil_div(n, bs);
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  return (unsigned)g;
}

}  // namespace

size_t scan_tmp_bytes(int64_t n, size_t elem) {
  size_t total = 0;
  int64_t m = n;
  while (m > STILE) {
    int64_t nb = ceil_div(m, STILE);
    total += (size_t)(((nb + 63) / 64) * 64) * elem;
    m = nb;
  }
  return total + 256;
}

void scan_u32(const uint32_t* in, uint32_t* out, int64_t n, void* tmp, hipStream_t st) { scan_impl<uint32_t>(in, out, n, tmp, st); }
void scan_u64(const uint64_t* in, uint64_t* out, int64_t n, void* tmp, hipStream_t st) { scan_impl<uint64_t>(in, out, n, tmp, st); }
void scan_i64(const int64_t* in, int64_t* out, int64_t n, void* tmp, hipStream_t st) { scan_impl<int64_t>(in, out, n, tmp, st); }

void key_or_and(const uint64_t* keys, int64_t n, uint64_t* out, uint64_t* part, hipStream_t st) {
  const unsigned g = n > 0 ? (grid_for(n, 256) > kOrAndBlocks ? (unsigned)kOrAndBlocks : grid_for(n, 256)) : 0;
  if (g > 0) hipLaunchKernelGGL(k_or_and_part, dim3(g), dim3(256), 0, st, keys, n, part);
  hipLaunchKernelGGL(k_or_and_final, dim3(1), dim3(256), 0, st, part, (int)g, out);
}

size_t radix_tmp_bytes(int64_t n) {
  int64_t nb = ceil_div(n > 0 ? n : 1, RTILE);
  return (size_t)(256 * nb) * 4 + scan_tmp_bytes(256 * nb, 4) + 256;
}

int radix_sort(uint64_t* k0, uint32_t* v0, uint64_t* k1, uint32_t* v1, int64_t n, int bit_lo, int bit_hi, void* tmp,
               hipStream_t st) {
  if (n <= 1 || bit_hi <= bit_lo) return 0;
  const int nb = (int)ceil_div(n, RTILE);
  uint32_t* hist = (uint32_t*)tmp;
  void* stmp = (void*)(hist + (((int64_t)256 * nb + 63) / 64) * 64);
  int cur = 0;
  for (int shift = (bit_lo / 8) * 8; shift < bit_hi; shift += 8) {
    const uint64_t* ki = cur ? k1 : k0;
    const uint32_t* vi = cur ? v1 : v0;
    uint64_t* ko = cur ? k0 : k1;
    uint32_t* vo = cur ? v0 : v1;
    hipLaunchKernelGGL(k_radix_hist, dim3(nb), dim3(RB), 0, st, ki, n, shift, hist, nb);
    scan_u32(hist, hist, (int64_t)256 * nb, stmp, st);
    hipLaunchKernelGGL(k_radix_scatter, dim3(nb), dim3(RB), 0, st, ki, vi, ko, vo, n, shift, (const uint32_t*)hist, nb);
    cur ^= 1;
  }
  return cur;
}

void fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_fill<uint32_t>, dim3(grid_for(n)), dim3(256), 0, st, p, v, n);
}
void fill_u64(uint64_t* p, uint64_t v, int64_t n, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_fill<uint64_t>, dim3(grid_for(n)), dim3(256), 0, st, p, v, n);
}
void iota_u32(uint32_t* p, int64_t n, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_iota, dim3(grid_for(n)), dim3(256), 0, st, p, n);
}
void gather_u64(const uint64_t* src, const uint32_t* idx, uint64_t* dst, int64_t n, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_gather64, dim3(grid_for(n)), dim3(256), 0, st, src, idx, dst, n);
}

}  // namespace w1
