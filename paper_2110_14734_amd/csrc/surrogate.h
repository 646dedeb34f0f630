// Learned surrogate (DeepSets network) for nearest-neighbour search over
// persistence diagrams: internal launchers and parameter layout.
#pragma once

#include "common.h"
#include "kernels.h"

namespace w1 {

// Network shape: phi 2 -> 128 -> 128 (ReLU after both), sum pooling,
// rho 128 -> 64 (linear).  Parameters, FP32, in one vector:
constexpr int DS_H = 128;
constexpr int DS_E = 64;
constexpr int DS_OFF_W1 = 0;                          // [128][2]  (birth, persistence)
constexpr int DS_OFF_B1 = DS_OFF_W1 + DS_H * 2;       // [128]
constexpr int DS_OFF_W2 = DS_OFF_B1 + DS_H;           // [128 out][128 in]
constexpr int DS_OFF_B2 = DS_OFF_W2 + DS_H * DS_H;    // [128]
constexpr int DS_OFF_W3 = DS_OFF_B2 + DS_H;           // [64][128]
constexpr int DS_OFF_B3 = DS_OFF_W3 + DS_E * DS_H;    // [64]
constexpr int DS_NPARAM = DS_OFF_B3 + DS_E;           // 25152

// Test functions of the dual lower bound used by the 1-NN search.
constexpr int NN_NSTATS = 33;

// MFMA operand images built from the FP32 parameters (BF16 bit patterns).
struct DsOperands {
  uint16_t* w1op;  // [8 k-blocks][64 lanes][8]
  uint16_t* w2op;  // [8 n-blocks][4 k-steps][64 lanes][8]
  uint16_t* w2t;   // [128 k][128 n] = bf16(W2[n][k])
};

// Per-row training outputs of the forward kernel (batch rows, each diagram
// padded to a multiple of 32 rows).
struct DsTrainRows {
  const int64_t* roff;  // [D + 1]
  int64_t rows;
  uint16_t* h1;         // [rows][128]
  uint16_t* h1t;        // [128][rows]
  uint32_t* m2;         // [rows][4] ReLU masks of layer 2 (lane-group packed)
  float2* xb;           // [rows] features as the network saw them (hi + lo)
  int32_t* cnt2;        // [D][128] active rows of each layer-2 unit
};

void ds_flags(const SegDesc* segs, int nseg, int64_t total, int dtype, uint32_t* flag, int32_t* err, hipStream_t st);
void ds_scatter(const SegDesc* segs, int nseg, int64_t total, int dtype, const uint32_t* flag, const uint32_t* pos,
                float2* X, hipStream_t st);
void ds_seg_starts(const SegDesc* segs, int nseg, const uint32_t* pos, int64_t total, int64_t* dstart,
                   hipStream_t st);
void ds_prep(const float* params, const DsOperands& op, hipStream_t st);
void ds_embed(const float2* X, const int64_t* dstart, const int32_t* dlist, int64_t D, const float* params,
              const DsOperands& op, float* pool, float* emb, const DsTrainRows* train, hipStream_t st);
void ds_loss(const float* emb, const int32_t* pa, const int32_t* pb, const double* w, int64_t P, float* gp,
             double* lpart, hipStream_t st);
void ds_demb(const float* gp, const int32_t* occ_start, const int32_t* occ, int64_t D, float* demb, hipStream_t st);
void ds_dW3(const float* demb, const float* pool, int64_t D, float* grad, hipStream_t st);
void ds_dpool(const float* demb, const float* params, int64_t D, float* dpool, hipStream_t st);
void ds_db2(const float* dpool, const int32_t* cnt2, int64_t D, float* grad, hipStream_t st);
void ds_dz2(const uint32_t* m2, const float* dpool, const int64_t* roff, int64_t D, int64_t rows, uint16_t* dz2,
            uint16_t* dz2t, hipStream_t st);
void ds_dlayer1(const float* dh1, const uint16_t* h1, const float2* xb, int64_t rows, int64_t slice, float* part,
                hipStream_t st);
void ds_gemm_nt(const uint16_t* A, const uint16_t* Bt, float* C, int64_t M, int64_t N, int64_t K, int64_t kslice,
                hipStream_t st);
void ds_sum_slices(const float* part, int64_t nz, int64_t n, float* out, hipStream_t st);
void ds_adam(float* w, const float* g, float* m1, float* m2, int64_t n, float lr, float beta1, float beta2, float eps,
             float bc1, float bc2, hipStream_t st);
void nn_stats(const SegDesc* segs, int nseg, int dtype, double* S, int32_t* err, hipStream_t st);
void ds_scores(const float* embq, int64_t nq, const float* embdb, int64_t m, float* out, hipStream_t st);

}  // namespace w1
