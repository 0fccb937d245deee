// Learned cost model (MLP 4 -> 64 -> 64 -> 1, FP32) used only to order and
// bin K-block work units; it never decides culling.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define FX_MLP_IN 4
#define FX_MLP_H 64
// packed parameter vector
#define FX_MLP_W1 0                                   // [H][IN]
#define FX_MLP_B1 (FX_MLP_W1 + FX_MLP_H * FX_MLP_IN)  // [H]
#define FX_MLP_W2 (FX_MLP_B1 + FX_MLP_H)              // [H][H]
#define FX_MLP_B2 (FX_MLP_W2 + FX_MLP_H * FX_MLP_H)   // [H]
#define FX_MLP_W3 (FX_MLP_B2 + FX_MLP_H)              // [H]
#define FX_MLP_B3 (FX_MLP_W3 + FX_MLP_H)              // scalar
#define FX_MLP_NPARAM (FX_MLP_B3 + 1)
// normalisation: mean[4], std[4], target mean, target std
#define FX_MLP_NNORM 10
// per-sample activations kept for the backward pass: h1, h2, dz2, dz1, dy, x[4]
#define FX_MLP_ACT (4 * FX_MLP_H + 1 + FX_MLP_IN)

void fx_launch_unit_features(const int* units, const long* ulh, long n_max, const long* bc_off, const long* cls_off,
                             int seg, const int* nprim, const double* qrow, float class_cost, float4* feat,
                             const long* feat_off, hipStream_t st);
void fx_launch_bound_cost(const float4* feat, const long* ulh, long n_max, float* out, hipStream_t st);
void fx_launch_qrow(const double* Qn, int S, double* qrow, hipStream_t st);
// ulh null: n_max samples; else ulh[1] - ulh[0] (read on the device) of at most n_max
void fx_launch_mlp_predict(const float* W, const float* norm, const float4* feat, const long* ulh, long n_max,
                           float* out, hipStream_t st);
void fx_mlp_backprop_grad(const float* W, const float* norm, const float4* feat, const float* target, const int* idx,
                          long n, float* act, float* loss_terms, float* grad, float* loss, hipStream_t st);
void fx_mlp_adam(float* W, const float* g, float* m, float* v, float lr, int t, hipStream_t st);
// blocks of the binned order for at most n_max units (bcount holds nbins * blocks counts)
long fx_bin_blocks(long n_max);
void fx_launch_bin_order(const float* cost, const long* ulh, long n_max, float top, float width, int nbins,
                         uint8_t* key, int* bcount, long* bpos, long* partial, long* total, int* order, hipStream_t st,
                         void (*scan)(const int*, long, long*, long*, long*, hipStream_t));
