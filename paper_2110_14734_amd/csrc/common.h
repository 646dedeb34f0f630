// Internal declarations of the w1approx HIP library (not part of the C-ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace w1 {

constexpr int WAVE = 64;

// ---------------------------------------------------------------- per pair --
// Per diagram-pair scalars, one array entry per pair, all in device memory.
// Counters are accumulated with atomics by the stage kernels.
struct PairArrays {
  int32_t* err;          // W1_E* code of the pair (0 = ok), set with atomicMin
  int64_t* nA;           // net A mass
  int64_t* nB;           // net B mass
  int32_t* locA;         // number of A locations (net > 0)
  int32_t* locB;         // number of B locations (net < 0)
  int64_t* loc_start;    // first location index
  int64_t* seg_lo;       // scratch: first index of the pair's run in a pair-major array
  int64_t* seg_hi;       // scratch: one past its last index (both zeroed before use)
  uint64_t* bmin;        // bounding box of locations, ordered bit patterns
  uint64_t* bmax;
  uint64_t* dmin;
  uint64_t* dmax;
  int32_t* beh;          // RWMD bucket side exponent
  int64_t* bx0;          // RWMD bucket grid origin (bucket units)
  int64_t* by0;
  int32_t* bnx;          // RWMD bucket grid size
  int32_t* bny;
  int64_t* bbase;        // first bucket id (scan over pairs)
  uint64_t* tmaxA;       // max RWMD term, bit pattern of a non-negative double
  uint64_t* tmaxB;
  uint64_t* sumA;        // fixed-point RWMD sums
  uint64_t* sumB;
  int32_t* FA;           // fixed-point shifts
  int32_t* FB;
  double* L;             // RWMD lower bound
  int32_t* e;            // grid exponent
  int64_t* m0;           // grid origin (cell units)
  int64_t* cell_start;   // first cell index of the pair
  int32_t* ncells;
  int64_t* item_start;   // first WSPD work item of the pair
  uint64_t* npairs;      // WSPD pairs of the pair
  uint64_t* pair_start;  // first output pair of the pair
  int32_t* costK;        // Euclidean network: costs in units of g 2^-costK
};

// ---------------------------------------------------------------- helpers --
__host__ __device__ inline uint64_t ordered_bits(uint64_t u) {
  return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}

__device__ inline uint64_t dbl_bits(double x) { return (uint64_t)__double_as_longlong(x); }
__device__ inline double bits_dbl(uint64_t u) { return __longlong_as_double((long long)u); }
__device__ inline double ordered_to_dbl(uint64_t o) {
  uint64_t u = (o >> 63) ? (o & 0x7fffffffffffffffull) : ~o;
  return bits_dbl(u);
}

__device__ inline int lane_id() { return (int)(threadIdx.x & (WAVE - 1)); }
__device__ inline uint64_t lanes_below() {
  int l = lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// Inclusive segmented reduction over a wave: a run is a maximal stretch of
// consecutive lanes with equal `key`; returns true on the last lane of each
// run, which then holds the run total in `v`.  Inactive lanes pass
// key = ~0u.  Equal keys separated by other keys are separate runs (each
// combine is bounded by the start of the lane's own run).
template <typename T, typename Op>
__device__ inline bool wave_seg_reduce(uint32_t key, T& v, Op op) {
  const int lane = lane_id();
  const uint32_t prev = __shfl_up(key, 1);
  int start = (lane == 0 || prev != key) ? lane : 0;
#pragma unroll
  for (int d = 1; d < WAVE; d <<= 1) {
    const int o = __shfl_up(start, d);
    if (lane >= d && o > start) start = o;
  }
#pragma unroll
  for (int d = 1; d < WAVE; d <<= 1) {
    T o = __shfl_up(v, d);
    if (lane - d >= start) v = op(v, o);
  }
  uint32_t nk = __shfl_down(key, 1);
  bool tail = (lane == WAVE - 1) || nk != key;
  return tail && key != ~0u;
}

// True when every thread of the block holds the same valid key (call once
// per kernel, from every thread).  Such a block is one run: after
// wave_seg_reduce the last lane of each wave holds its wave's total, and
// block_total combines them, so one atomic per block replaces one per wave.
__device__ inline bool block_single_key(uint32_t key) {
  __shared__ uint32_t s_k0;
  if (threadIdx.x == 0) s_k0 = key;
  __syncthreads();
  const uint32_t k0 = s_k0;
  return __syncthreads_and(key == k0 && k0 != ~0u) != 0;
}

template <typename T, typename Op>
__device__ inline T block_total(T v, Op op) {  // 256-thread blocks, after wave_seg_reduce of one run
  __shared__ T s[4];
  if (lane_id() == WAVE - 1) s[threadIdx.x / WAVE] = v;
  __syncthreads();
  const T r = op(op(s[0], s[1]), op(s[2], s[3]));
  __syncthreads();
  return r;
}

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ------------------------------------------------------------- primitives --
// Exclusive scan of n values (in place allowed).  `tmp` needs scan_tmp_bytes.
size_t scan_tmp_bytes(int64_t n, size_t elem);
void scan_u32(const uint32_t* in, uint32_t* out, int64_t n, void* tmp, hipStream_t st);
void scan_u64(const uint64_t* in, uint64_t* out, int64_t n, void* tmp, hipStream_t st);
void scan_i64(const int64_t* in, int64_t* out, int64_t n, void* tmp, hipStream_t st);

// OR and AND of n keys into out[0], out[1] (device).
// out[0] = OR, out[1] = AND of the n keys (0 and ~0 for n = 0); part holds
// 2 kOrAndBlocks words of scratch.
constexpr int kOrAndBlocks = 1024;
void key_or_and(const uint64_t* keys, int64_t n, uint64_t* out, uint64_t* part, hipStream_t st);

// Stable LSD radix sort of (key, value) by bits [bit_lo, bit_hi), 8-bit
// digits.  Buffers k0/v0 hold the input; k1/v1 are scratch of equal size.
// Returns 0 if the result is in (k0, v0), 1 if in (k1, v1).
size_t radix_tmp_bytes(int64_t n);
int radix_sort(uint64_t* k0, uint32_t* v0, uint64_t* k1, uint32_t* v1, int64_t n, int bit_lo, int bit_hi,
               void* tmp, hipStream_t st);

void fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t st);
void fill_u64(uint64_t* p, uint64_t v, int64_t n, hipStream_t st);
void iota_u32(uint32_t* p, int64_t n, hipStream_t st);
void gather_u64(const uint64_t* src, const uint32_t* idx, uint64_t* dst, int64_t n, hipStream_t st);

}  // namespace w1
