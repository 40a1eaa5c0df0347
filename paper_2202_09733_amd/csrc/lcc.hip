// Learned coarse correction for the p-multigrid preconditioner (gfx950).
//
// An element-local, bias-free ReLU network N (in -> H -> H -> out) refines
// the element-local coarse EJ step C1 = B1^{-1} Gamma d: it reads C1 on the
// element and on its 2 dim face neighbours, and the element's
// (log) sizes, and returns what a deeper coarse solve adds to C1; together
// they replace the coarse smoothing sweeps of the V-cycle.  The C1 inputs are
// standardised per variable (fixed scales from the training data) and divided
// by their per-element norm s; the output is multiplied back by s, so the
// correction is exactly positive-homogeneous in the defect, and it is made
// odd by evaluating N on (+x, g) and (-x, g), g the geometry entries:
// C = C1 + tau s (N(x/s, g) - N(-x/s, g)) / 2.
//
// Every product runs on BF16-input MFMA (v_mfma_f32_16x16x32_bf16) with FP32
// accumulation: one kernel computes C = A B^T for K-contiguous row-major A
// [M x K] and B [N x K] with a fused epilogue (FP32 store, ReLU to BF16, or
// ReLU-mask to BF16 for the backward pass).  Training keeps FP32 master
// weights updated by Adam and BF16 copies for the products.
#include <cmath>
#include <cstring>
#include <vector>

#include "lcc.hpp"

namespace frpmg {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kTile = 32;  // workgroup tile (M and N); 4 waves of 16 x 16

__device__ __forceinline__ __bf16 to_bf(float x) { return (__bf16)x; }
__device__ __forceinline__ float from_bf(__bf16 x) { return (float)x; }

// C[m][n] = sum_k A[m][k] B[n][k]; A: M x K (lda), B: N x K (ldb), K % 32 == 0,
// M % 32 == 0, N % 32 == 0 (callers pad).  Lane l of a wave holds
// A[row l%16][k 8(l/16)..+7], B[col l%16][k 8(l/16)..+7] and returns
// C[row 4(l/16)+i][col l%16], i = 0..3.
template <int EP>
__global__ void __launch_bounds__(256) k_gemm_nt(int M, int N, int K, const __bf16 *__restrict__ A, int lda,
                                                 const __bf16 *__restrict__ B, int ldb, float *__restrict__ Cf,
                                                 __bf16 *__restrict__ Cb, int ldc, const __bf16 *__restrict__ mask,
                                                 float alpha) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m0 = blockIdx.y * kTile + (wave >> 1) * 16;
    const int n0 = blockIdx.x * kTile + (wave & 1) * 16;
    const int r = lane & 15, g = lane >> 4;
    const __bf16 *pa = A + (size_t)(m0 + r) * lda + 8 * g;
    const __bf16 *pb = B + (size_t)(n0 + r) * ldb + 8 * g;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int k = 0; k < K; k += 32) {
        const bf16x8 a = *reinterpret_cast<const bf16x8 *>(pa + k);
        const bf16x8 b = *reinterpret_cast<const bf16x8 *>(pb + k);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int row = m0 + 4 * g + i, col = n0 + r;
        const float v = alpha * acc[i];
        const size_t idx = (size_t)row * ldc + col;
        if (EP == LCC_EP_F32) {
            Cf[idx] = v;
        } else if (EP == LCC_EP_RELU) {
            Cb[idx] = to_bf(v > 0.f ? v : 0.f);
        } else {  // ReLU derivative mask from the forward activation
            Cb[idx] = to_bf(from_bf(mask[idx]) > 0.f ? v : 0.f);
        }
    }
}

__global__ void k_transpose_bf(int rows, int cols, const __bf16 *__restrict__ in, int ldi, __bf16 *__restrict__ out,
                               int ldo) {
    __shared__ __bf16 tile[32][33];
    const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
    for (int j = ty; j < 32; j += 8) {
        const int rr = by + j, cc = bx + tx;
        tile[j][tx] = (rr < rows && cc < cols) ? in[(size_t)rr * ldi + cc] : to_bf(0.f);
    }
    __syncthreads();
    for (int j = ty; j < 32; j += 8) {
        const int rr = bx + j, cc = by + tx;  // out[cc_in][rr_in]
        if (rr < cols && cc < rows) out[(size_t)rr * ldo + cc] = tile[tx][j];
    }
}

__global__ void k_f32_to_bf(size_t n, const float *__restrict__ a, __bf16 *__restrict__ b) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) b[i] = to_bf(a[i]);
}

// Feature rows of one level-1 defect field d (layout [nv][Np1][Ne]):
// [own d (nv Np1) | for each axis a: the -a neighbour's d, then the +a
//  neighbour's d (nv Np1 each)] / sigma_v, zero padded to ld, then divided by
// the row norm s (s = 0: zero row).
// sign_rows: rows Ne..2Ne-1 receive the negated row (odd evaluation).
// After the normalised defect part come dim geometry entries
// ln(h_a(k) / max_a h), which do not scale with the defect.
// One 64-lane wavefront per element row: each lane forms the entries
// j = lane, lane + 64, ..., the row norm is a wavefront reduction.
constexpr int kFeatPerLane = 16;  // rows up to 64 x 16 = 1024 entries

template <int DIM>
__global__ void __launch_bounds__(256) k_features(int Ne, int nx, int ny, int P, const double *__restrict__ d,
                                                  const float *__restrict__ in_scale, int ld, int nin,
                                                  float *__restrict__ Xf, __bf16 *__restrict__ Xb,
                                                  float *__restrict__ srow, int both_signs, MeshK mesh, double hx,
                                                  double hy, double hz) {
    const int k = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (k >= Ne) return;
    const int nv = DIM + 2;
    const int Np = (DIM == 2) ? P * P : P * P * P;
    const int nblk = nv * Np;
    const int ix = k % nx, iy = (k / nx) % ny, iz = k / (nx * ny);
    const int nz = Ne / (nx * ny);
    const int ndef = nin - DIM;  // defect entries
    float vals[kFeatPerLane];
    double ss = 0.0;
#pragma unroll
    for (int u = 0; u < kFeatPerLane; ++u) {
        const int j = lane + 64 * u;
        float x = 0.f;
        if (j < ndef) {
            const int part = j / nblk, rem = j - part * nblk;
            const int v = rem / Np, i = rem - v * Np;
            int kel = k;
            if (part > 0) {
                // part 1 + 2a + side: side 0 the -a neighbour, side 1 the +a neighbour
                const int a = (part - 1) >> 1;
                const int sgn = ((part - 1) & 1) ? 1 : -1;
                int jx = ix, jy = iy, jz = iz;
                if (a == 0) jx = (ix + sgn + nx) % nx;
                if (a == 1) jy = (iy + sgn + ny) % ny;
                if (a == 2) jz = (iz + sgn + nz) % nz;
                kel = jx + nx * (jy + ny * jz);
            }
            x = (float)(d[((size_t)v * Np + i) * Ne + kel] / in_scale[v]);
            ss += (double)x * x;
        }
        vals[u] = x;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) ss += __shfl_xor(ss, off, 64);
    const float sn = (float)sqrt(ss);
    const float inv = sn > 0.f ? 1.f / sn : 0.f;
    const int ic[3] = {ix, iy, iz};
    const double hmax[3] = {hx, hy, hz};
    float *row = Xf + (size_t)k * ld;
#pragma unroll
    for (int u = 0; u < kFeatPerLane; ++u) {
        const int j = lane + 64 * u;
        if (j >= ld) break;
        float x = 0.f, xm = 0.f;
        if (j < ndef) {
            x = vals[u] * inv;
            xm = -x;
        } else if (j < nin) {
            const int a = j - ndef;
            x = (float)log((2.0 / mesh.inv2h[a][ic[a]]) / hmax[a]);
            xm = x;
        }
        row[j] = x;
        Xb[(size_t)k * ld + j] = to_bf(x);
        if (both_signs) Xb[(size_t)(Ne + k) * ld + j] = to_bf(xm);
    }
    if (lane == 0) srow[k] = sn;
}

// Target rows: C (layout [nv][Np1][Ne]) / tau_v / s, zero padded.
__global__ void k_targets(int Ne, int nv, int Np, const double *__restrict__ C, const float *__restrict__ out_scale,
                          const float *__restrict__ srow, int ld, float *__restrict__ T) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= Ne) return;
    const float s = srow[k];
    const float inv = s > 0.f ? 1.f / s : 0.f;
    for (int j = 0; j < ld; ++j) {
        float t = 0.f;
        if (j < nv * Np) {
            const int v = j / Np, i = j % Np;
            t = (float)(C[((size_t)v * Np + i) * Ne + k] / out_scale[v]) * inv;
        }
        T[(size_t)k * ld + j] = t;
    }
}

// C[v][i][k] = tau_v s_k (Y[k][j] - Y[Ne + k][j]) / 2,  j = v Np + i
__global__ void k_output(int Ne, int nv, int Np, const float *__restrict__ Y, int ld, const float *__restrict__ srow,
                         const float *__restrict__ out_scale, double *__restrict__ C) {
    const size_t total = (size_t)nv * Np * Ne;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += stride) {
        const int k = (int)(idx % Ne);
        const int j = (int)(idx / Ne);  // v * Np + i
        const int v = j / Np;
        const float y = 0.5f * (Y[(size_t)k * ld + j] - Y[(size_t)(Ne + k) * ld + j]);
        C[idx] = (double)out_scale[v] * (double)srow[k] * (double)y;
    }
}

// copy selected rows (every stride-th element starting at offset) into the
// harvest buffers at position base
__global__ void k_harvest_rows(int Ne, int stride, int offset, int base, int cap, int ldx, int ldt,
                               const float *__restrict__ Xf, const float *__restrict__ Tf, float *__restrict__ HX,
                               float *__restrict__ HT) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int k = offset + t * stride;
    if (k >= Ne) return;
    const int dst = base + t;
    if (dst >= cap) return;
    for (int j = 0; j < ldx; ++j) HX[(size_t)dst * ldx + j] = Xf[(size_t)k * ldx + j];
    for (int j = 0; j < ldt; ++j) HT[(size_t)dst * ldt + j] = Tf[(size_t)k * ldt + j];
}

// batch gather: rows idx[b] of the harvest buffers -> X (bf16), T (f32).
// flip = 1: odd batch positions get the sign-flipped pair (-x, -t) with the
// geometry entries [ndef, nin) unchanged, so the network sees both signs of
// the defect that the odd evaluation N(x) - N(-x) uses.
__global__ void k_gather_batch(int B, const int *__restrict__ idx, int ldx, int ldt, int ndef, int flip,
                               const float *__restrict__ HX, const float *__restrict__ HT, __bf16 *__restrict__ Xb,
                               float *__restrict__ Tb) {
    const int b = blockIdx.x;
    const int r = idx[b];
    const float sg = (flip && (b & 1)) ? -1.f : 1.f;
    for (int j = threadIdx.x; j < ldx; j += blockDim.x) {
        const float x = HX[(size_t)r * ldx + j];
        Xb[(size_t)b * ldx + j] = to_bf(j < ndef ? sg * x : x);
    }
    for (int j = threadIdx.x; j < ldt; j += blockDim.x) Tb[(size_t)b * ldt + j] = sg * HT[(size_t)r * ldt + j];
}

// dY = (Y - T) / B as bf16 (padded columns carry zero targets and weights);
// loss partial sums of 0.5 (Y - T)^2 / B per block
__global__ void __launch_bounds__(256) k_loss_grad(int B, int ld, int nout, const float *__restrict__ Y,
                                                   const float *__restrict__ T, __bf16 *__restrict__ dY,
                                                   double *__restrict__ partial) {
    __shared__ double red[4];
    const size_t total = (size_t)B * ld;
    double acc = 0.0;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
        const int j = (int)(i % ld);
        const float e = (j < nout) ? (Y[i] - T[i]) : 0.f;
        dY[i] = to_bf(e / B);
        acc += 0.5 * (double)e * e / B;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ void k_sum_small(int n, const double *__restrict__ p, double *__restrict__ out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < n; ++i) s += p[i];
        *out = s;
    }
}

__global__ void k_adam(size_t n, float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, __bf16 *__restrict__ wb, float lr, float b1, float b2, float eps, float c1,
                       float c2) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
        w[i] = wi;
        wb[i] = to_bf(wi);
    }
}

unsigned gridN(size_t n) {
    size_t b = (n + 255) / 256;
    if (b > 4096) b = 4096;
    return (unsigned)(b ? b : 1);
}

}  // namespace

hipError_t lcc_gemm(int ep, int M, int N, int K, const __bf16 *A, int lda, const __bf16 *B, int ldb, float *Cf,
                    __bf16 *Cb, int ldc, const __bf16 *mask, float alpha, hipStream_t s) {
    if (M % kTile || N % kTile || K % 32) return hipErrorInvalidValue;
    dim3 grid(N / kTile, M / kTile);
    if (ep == LCC_EP_F32)
        hipLaunchKernelGGL(k_gemm_nt<LCC_EP_F32>, grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, Cf, Cb, ldc, mask,
                           alpha);
    else if (ep == LCC_EP_RELU)
        hipLaunchKernelGGL(k_gemm_nt<LCC_EP_RELU>, grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, Cf, Cb, ldc, mask,
                           alpha);
    else
        hipLaunchKernelGGL(k_gemm_nt<LCC_EP_MASK>, grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, Cf, Cb, ldc, mask,
                           alpha);
    return hipGetLastError();
}

hipError_t lcc_transpose(int rows, int cols, const __bf16 *in, int ldi, __bf16 *out, int ldo, hipStream_t s) {
    dim3 grid((cols + 31) / 32, (rows + 31) / 32);
    hipLaunchKernelGGL(k_transpose_bf, grid, dim3(256), 0, s, rows, cols, in, ldi, out, ldo);
    return hipGetLastError();
}

hipError_t lcc_to_bf(size_t n, const float *a, __bf16 *b, hipStream_t s) {
    hipLaunchKernelGGL(k_f32_to_bf, dim3(gridN(n)), dim3(256), 0, s, n, a, b);
    return hipGetLastError();
}

hipError_t lcc_features(const frpmg_ctx *ctx, const double *d, const Lcc &L, float *Xf, __bf16 *Xb, float *srow,
                        int both_signs, hipStream_t s) {
    const int Ne = ctx->mesh.Ne;
    const Level &C = ctx->lv[1];
    if (L.nin_pad > 64 * kFeatPerLane) return hipErrorInvalidValue;
    dim3 grid((Ne + 3) / 4);  // four elements (wavefronts) per workgroup
    if (ctx->dim == 2)
        hipLaunchKernelGGL(k_features<2>, grid, dim3(256), 0, s, Ne, ctx->mesh.n[0], ctx->mesh.n[1], C.P, d,
                           L.in_scale, L.nin_pad, L.nin, Xf, Xb, srow, both_signs, ctx->mesh, L.hmax[0], L.hmax[1],
                           L.hmax[2]);
    else
        hipLaunchKernelGGL(k_features<3>, grid, dim3(256), 0, s, Ne, ctx->mesh.n[0], ctx->mesh.n[1], C.P, d,
                           L.in_scale, L.nin_pad, L.nin, Xf, Xb, srow, both_signs, ctx->mesh, L.hmax[0], L.hmax[1],
                           L.hmax[2]);
    return hipGetLastError();
}

hipError_t lcc_targets(const frpmg_ctx *ctx, const double *Cc, const Lcc &L, const float *srow, float *T,
                       hipStream_t s) {
    const int Ne = ctx->mesh.Ne;
    hipLaunchKernelGGL(k_targets, dim3((Ne + 127) / 128), dim3(128), 0, s, Ne, ctx->nv, ctx->lv[1].Np, Cc,
                       L.out_scale, srow, L.nout_pad, T);
    return hipGetLastError();
}

hipError_t lcc_output(const frpmg_ctx *ctx, const Lcc &L, const float *Y, const float *srow, double *Cc,
                      hipStream_t s) {
    const int Ne = ctx->mesh.Ne;
    const size_t total = (size_t)ctx->nv * ctx->lv[1].Np * Ne;
    hipLaunchKernelGGL(k_output, dim3(gridN(total)), dim3(256), 0, s, Ne, ctx->nv, ctx->lv[1].Np, Y, L.nout_pad, srow,
                       L.out_scale, Cc);
    return hipGetLastError();
}

hipError_t lcc_harvest_rows(const Lcc &L, int Ne, int stride, int offset, int base, const float *Xf, const float *Tf,
                            hipStream_t s) {
    const int n = (Ne - offset + stride - 1) / stride;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_harvest_rows, dim3((n + 127) / 128), dim3(128), 0, s, Ne, stride, offset, base, L.cap,
                       L.nin_pad, L.nout_pad, Xf, Tf, L.HX, L.HT);
    return hipGetLastError();
}

hipError_t lcc_gather_batch(const Lcc &L, int B, const int *idx, __bf16 *Xb, float *Tb, int flip, hipStream_t s) {
    const int ndef = L.nin - L.ngeo;
    hipLaunchKernelGGL(k_gather_batch, dim3(B), dim3(128), 0, s, B, idx, L.nin_pad, L.nout_pad, ndef, flip, L.HX,
                       L.HT, Xb, Tb);
    return hipGetLastError();
}

hipError_t lcc_loss_grad(int B, int ld, int nout, const float *Y, const float *T, __bf16 *dY, double *partial,
                         double *loss, hipStream_t s) {
    const int nblk = 64;
    hipLaunchKernelGGL(k_loss_grad, dim3(nblk), dim3(256), 0, s, B, ld, nout, Y, T, dY, partial);
    hipLaunchKernelGGL(k_sum_small, dim3(1), dim3(64), 0, s, nblk, partial, loss);
    return hipGetLastError();
}

hipError_t lcc_adam(size_t n, float *w, const float *g, float *m, float *v, __bf16 *wb, float lr, float b1, float b2,
                    float eps, int step, hipStream_t s) {
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3(gridN(n)), dim3(256), 0, s, n, w, g, m, v, wb, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

}  // namespace frpmg
