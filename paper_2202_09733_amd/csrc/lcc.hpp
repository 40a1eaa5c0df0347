// Learned coarse correction: device buffers and kernel launchers (internal).
#pragma once

#include "internal.hpp"

namespace frpmg {

enum { LCC_EP_F32 = 0, LCC_EP_RELU = 1, LCC_EP_MASK = 2 };

// Adam hyper-parameters (Kingma and Ba's defaults)
constexpr float kAdamB1 = 0.9f, kAdamB2 = 0.999f, kAdamEps = 1e-8f;

struct Lcc {
    int nin = 0, nin_pad = 0, nh = 256, nout = 0, nout_pad = 0, ngeo = 0;
    int wrows[3] = {0, 0, 0}, wcols[3] = {0, 0, 0};
    float *W[3] = {nullptr, nullptr, nullptr};   // FP32 masters
    float *G[3] = {nullptr, nullptr, nullptr};   // gradients
    float *Mo[3] = {nullptr, nullptr, nullptr};  // Adam first moments
    float *Vo[3] = {nullptr, nullptr, nullptr};  // Adam second moments
    __bf16 *Wb[3] = {nullptr, nullptr, nullptr};   // BF16 copies
    __bf16 *WbT[3] = {nullptr, nullptr, nullptr};  // BF16 transposes (backward)
    float *in_scale = nullptr, *out_scale = nullptr;  // device [nv]
    float h_in_scale[5] = {0, 0, 0, 0, 0}, h_out_scale[5] = {0, 0, 0, 0, 0};
    int scales_set = 0;
    double hmax[3] = {1.0, 1.0, 1.0};  // largest element width per axis
    int weights_set = 0;
    // harvesting
    int harvesting = 0, cap = 0, count = 0, stride = 8, target_sweeps = 8, cycle = 0;
    float *HX = nullptr, *HT = nullptr;
    // inference / harvest per-element buffers
    int Mpad = 0;
    float *Xf = nullptr, *Tf = nullptr, *srow = nullptr, *Y = nullptr;
    __bf16 *Xb = nullptr, *H1 = nullptr, *H2 = nullptr;
    double *dtmp = nullptr, *Cuse = nullptr;
    // training buffers
    int B = 0;
    __bf16 *bX = nullptr, *bXT = nullptr, *bH1 = nullptr, *bH1T = nullptr, *bH2 = nullptr, *bH2T = nullptr;
    __bf16 *bdY = nullptr, *bdYT = nullptr, *bdH2 = nullptr, *bdH2T = nullptr, *bdH1 = nullptr, *bdH1T = nullptr;
    float *bY = nullptr, *bT = nullptr;
    int *perm = nullptr;
    size_t perm_cap = 0;
    double *lpart = nullptr, *lval = nullptr;
    int adam_step = 0;
};

hipError_t lcc_gemm(int ep, int M, int N, int K, const __bf16 *A, int lda, const __bf16 *B, int ldb, float *Cf,
                    __bf16 *Cb, int ldc, const __bf16 *mask, float alpha, hipStream_t s);
hipError_t lcc_transpose(int rows, int cols, const __bf16 *in, int ldi, __bf16 *out, int ldo, hipStream_t s);
hipError_t lcc_to_bf(size_t n, const float *a, __bf16 *b, hipStream_t s);
hipError_t lcc_features(const frpmg_ctx *ctx, const double *d, const Lcc &L, float *Xf, __bf16 *Xb, float *srow,
                        int both_signs, hipStream_t s);
hipError_t lcc_targets(const frpmg_ctx *ctx, const double *Cc, const Lcc &L, const float *srow, float *T,
                       hipStream_t s);
hipError_t lcc_output(const frpmg_ctx *ctx, const Lcc &L, const float *Y, const float *srow, double *Cc,
                      hipStream_t s);
hipError_t lcc_harvest_rows(const Lcc &L, int Ne, int stride, int offset, int base, const float *Xf, const float *Tf,
                            hipStream_t s);
hipError_t lcc_gather_batch(const Lcc &L, int B, const int *idx, __bf16 *Xb, float *Tb, int flip, hipStream_t s);
hipError_t lcc_loss_grad(int B, int ld, int nout, const float *Y, const float *T, __bf16 *dY, double *partial,
                         double *loss, hipStream_t s);
hipError_t lcc_adam(size_t n, float *w, const float *g, float *m, float *v, __bf16 *wb, float lr, float b1, float b2,
                    float eps, int step, hipStream_t s);

}  // namespace frpmg
