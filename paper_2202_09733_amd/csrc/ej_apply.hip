// Element-Jacobi apply on gfx950: y = beta y + alpha B^{-1} r for every
// element at once with the stored inverse blocks (Sec. 2.2, element-Jacobi
// preconditioner; Sec. 3.2, EJ smoother).  A batched GEMV that streams the
// inverses once from HBM: each lane owns R consecutive rows of one block and
// reads them with one 16-byte load per block column (FP64 R = 2, FP32 and
// BF16 R = 4), accumulating in FP64.  This is the HBM-bound kernel of the
// preconditioner.
#include "internal.hpp"

namespace frpmg {

namespace {

constexpr int kApplyThreads = 256;

// Loads of the stored inverse, with or without the non-temporal hint (NT).
// An inverse larger than the 256 MB last-level cache is streamed from HBM on
// every apply: the hint keeps it from displacing r and y, and the 26.8 GB
// 32^3 p = 3 stream runs at 6.2 TB/s instead of 4.9 (64x64 p = 4, 328 MB: 55
// instead of 57 us).  A smaller one (the FP32/BF16 64x64 p = 4 inverses, every
// coarse level of that mesh) is served from that cache by the V-cycle's
// repeated applies, which the hint would defeat (BF16: 17 -> 20 us).
typedef double nt_d2 __attribute__((ext_vector_type(2)));
typedef float nt_f4 __attribute__((ext_vector_type(4)));

template <bool NT, typename U>
__device__ __forceinline__ U ld(const U *p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}

__device__ __forceinline__ double bf16_bits(unsigned int h) { return (double)__uint_as_float(h << 16); }

template <typename T, int R, bool NT>
struct VecLoad;
template <bool NT>
struct VecLoad<double, 1, NT> {
    __device__ static void get(const double *p, double *o) { o[0] = ld<NT>(p); }
};
template <bool NT>
struct VecLoad<double, 2, NT> {
    __device__ static void get(const double *p, double *o) {
        const nt_d2 v = ld<NT>(reinterpret_cast<const nt_d2 *>(p));
        o[0] = v.x;
        o[1] = v.y;
    }
};
template <bool NT>
struct VecLoad<float, 1, NT> {
    __device__ static void get(const float *p, double *o) { o[0] = ld<NT>(p); }
};
template <bool NT>
struct VecLoad<float, 4, NT> {
    __device__ static void get(const float *p, double *o) {
        const nt_f4 v = ld<NT>(reinterpret_cast<const nt_f4 *>(p));
        o[0] = v.x;
        o[1] = v.y;
        o[2] = v.z;
        o[3] = v.w;
    }
};

// BF16 entries are loaded as their bit patterns (the upper half of an FP32)
template <bool NT>
struct VecLoad<__bf16, 1, NT> {
    __device__ static void get(const __bf16 *p, double *o) {
        o[0] = bf16_bits(ld<NT>(reinterpret_cast<const unsigned short *>(p)));
    }
};
template <bool NT>
struct VecLoad<__bf16, 4, NT> {
    __device__ static void get(const __bf16 *p, double *o) {
        const unsigned long long u = ld<NT>(reinterpret_cast<const unsigned long long *>(p));
        o[0] = bf16_bits((unsigned int)(u & 0xffffu));
        o[1] = bf16_bits((unsigned int)((u >> 16) & 0xffffu));
        o[2] = bf16_bits((unsigned int)((u >> 32) & 0xffffu));
        o[3] = bf16_bits((unsigned int)(u >> 48));
    }
};

// y[row][k] = beta y + alpha sum_j Binv_k[row][j] r[j][k], Binv column-major.
// Each lane owns R consecutive rows of one block and streams the block
// column by column with one wide load per column (R = 2 for FP64, 4 for FP32
// and BF16 storage), so a wavefront reads whole contiguous column segments.
// Where few long per-lane column loops would leave the chip poorly balanced,
// the columns are split into S contiguous ranges on S lane groups, whose
// partial sums meet in LDS and are added in range order.  With a column placement (blocked inversion), stored column j
// multiplies r[cols[j]]; the gather happens while r is staged in LDS.
template <typename T, int R, bool NT>
__global__ void __launch_bounds__(kApplyThreads) k_ej_apply(int nb, int Ne, int epb, int S,
                                                            const T *__restrict__ inv,
                                                            const int *__restrict__ cols,
                                                            const double *__restrict__ r, double alpha,
                                                            double beta, const double *yin, Scal scale,
                                                            double *y) {
    extern __shared__ double s_r[];  // [epb][nb], then the partial sums [epb][S][nb] when S > 1
    const int k0 = xcd_block(blockIdx.x, gridDim.x) * epb;  // r and y lines stay within one XCD
    const int ne = min(epb, Ne - k0);
    for (int t = threadIdx.x; t < epb * nb; t += blockDim.x) {
        const int e = t / nb, j = t - e * nb;
        double v = 0.0;
        if (e < ne) {
            const int jr = cols ? cols[(size_t)(k0 + e) * nb + j] : j;
            v = r[(size_t)jr * Ne + k0 + e];
        }
        s_r[t] = v;
    }
    __syncthreads();
    const int tpe = nb / R;  // row groups per block
    const int lpe = tpe * S;
    const int e = threadIdx.x / lpe;
    const int rem = threadIdx.x - e * lpe;
    const int sg = rem / tpe;
    const int row = (rem - sg * tpe) * R;
    const bool active = e < ne;
    const int cs = (nb + S - 1) / S;
    const int j0 = sg * cs, j1 = min(nb, j0 + cs);
    double acc[R];
#pragma unroll
    for (int q = 0; q < R; ++q) acc[q] = 0.0;
    if (active) {
        const int k = k0 + e;
        const T *col = inv + (size_t)k * nb * nb + row;
        const double *rv = s_r + e * nb;
        int j = j0;
        if constexpr (sizeof(T) < sizeof(double)) {
            // narrow storage: eight column loads in flight per lane (fewer
            // lanes per block; measured 18.9 -> 17.1 us for 4096 BF16 blocks
            // of 100^2, no change in FP64)
            for (; j + 8 <= j1; j += 8) {
                double v0[R], v1[R], v2[R], v3[R], v4[R], v5[R], v6[R], v7[R];
                VecLoad<T, R, NT>::get(col + (size_t)j * nb, v0);
                VecLoad<T, R, NT>::get(col + (size_t)(j + 1) * nb, v1);
                VecLoad<T, R, NT>::get(col + (size_t)(j + 2) * nb, v2);
                VecLoad<T, R, NT>::get(col + (size_t)(j + 3) * nb, v3);
                VecLoad<T, R, NT>::get(col + (size_t)(j + 4) * nb, v4);
                VecLoad<T, R, NT>::get(col + (size_t)(j + 5) * nb, v5);
                VecLoad<T, R, NT>::get(col + (size_t)(j + 6) * nb, v6);
                VecLoad<T, R, NT>::get(col + (size_t)(j + 7) * nb, v7);
#pragma unroll
                for (int q = 0; q < R; ++q)
                    acc[q] += ((v0[q] * rv[j] + v1[q] * rv[j + 1]) + (v2[q] * rv[j + 2] + v3[q] * rv[j + 3])) +
                              ((v4[q] * rv[j + 4] + v5[q] * rv[j + 5]) + (v6[q] * rv[j + 6] + v7[q] * rv[j + 7]));
            }
        }
        for (; j + 4 <= j1; j += 4) {
            double v0[R], v1[R], v2[R], v3[R];
            VecLoad<T, R, NT>::get(col + (size_t)j * nb, v0);
            VecLoad<T, R, NT>::get(col + (size_t)(j + 1) * nb, v1);
            VecLoad<T, R, NT>::get(col + (size_t)(j + 2) * nb, v2);
            VecLoad<T, R, NT>::get(col + (size_t)(j + 3) * nb, v3);
            const double x0 = rv[j], x1 = rv[j + 1], x2 = rv[j + 2], x3 = rv[j + 3];
#pragma unroll
            for (int q = 0; q < R; ++q) acc[q] += (v0[q] * x0 + v1[q] * x1) + (v2[q] * x2 + v3[q] * x3);
        }
        for (; j < j1; ++j) {
            double v0[R];
            VecLoad<T, R, NT>::get(col + (size_t)j * nb, v0);
#pragma unroll
            for (int q = 0; q < R; ++q) acc[q] += v0[q] * rv[j];
        }
    }
    if (S > 1) {
        double *part = s_r + epb * nb;  // [epb][S][nb]
        if (active) {
#pragma unroll
            for (int q = 0; q < R; ++q) part[((size_t)e * S + sg) * nb + row + q] = acc[q];
        }
        __syncthreads();
        if (!active || sg != 0) return;
#pragma unroll
        for (int q = 0; q < R; ++q) {
            double t = part[((size_t)e * S) * nb + row + q];
            for (int s2 = 1; s2 < S; ++s2) t += part[((size_t)e * S + s2) * nb + row + q];
            acc[q] = t;
        }
    }
    if (!active) return;
    const int k = k0 + e;
    const double sc = sval(scale);
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const size_t idx = (size_t)(row + q) * Ne + k;
        y[idx] = sc * ((beta == 0.0) ? alpha * acc[q] : beta * yin[idx] + alpha * acc[q]);
    }
}

// Column ranges per block.  FP64 storage on fewer than 256k lanes (4
// wavefronts per SIMD) takes two ranges: at 4096 blocks of 100^2 that turns
// 820 workgroups of 100-column loops into 2048 of 50 (66.5 -> 62.5 us).
// Measured not to pay for the 36^2 blocks or for FP32/BF16 storage.
template <typename T>
int apply_split(int nb, int tpe, int Ne) {
    return (sizeof(T) == 8 && (size_t)Ne * tpe < (256u << 10) && nb >= 64 && 2 * tpe <= kApplyThreads) ? 2 : 1;
}

// inverses above this size take the non-temporal loads (see VecLoad)
constexpr size_t kStreamedInverse = size_t(192) << 20;

template <typename T, int R>
hipError_t launch_apply(const Level &L, int Ne, const double *r, double alpha, double beta, const double *yin,
                        Scal scale, double *y, hipStream_t s) {
    const int nb = L.nb;
    const int tpe = nb / R;
    if (tpe > kApplyThreads) return hipErrorInvalidValue;
    const int S = apply_split<T>(nb, tpe, Ne);
    const int lpe = tpe * S;
    const int epb = (lpe >= kApplyThreads) ? 1 : kApplyThreads / lpe;
    const size_t lds = (size_t)epb * nb * (S > 1 ? 1 + S : 1) * sizeof(double);
    dim3 grid((Ne + epb - 1) / epb);
    dim3 block((epb * lpe + 63) / 64 * 64);  // whole wavefronts, none without a block row
    if ((size_t)Ne * nb * nb * sizeof(T) > kStreamedInverse)
        hipLaunchKernelGGL((k_ej_apply<T, R, true>), grid, block, lds, s, nb, Ne, epb, S, (const T *)L.inv,
                           L.inv_cols, r, alpha, beta, yin, scale, y);
    else
        hipLaunchKernelGGL((k_ej_apply<T, R, false>), grid, block, lds, s, nb, Ne, epb, S, (const T *)L.inv,
                           L.inv_cols, r, alpha, beta, yin, scale, y);
    return hipGetLastError();
}

}  // namespace

hipError_t ej_apply_ex(const frpmg_ctx *ctx, int level, const double *r, double alpha, double beta,
                       const double *yin, Scal scale, double *y, hipStream_t s) {
    const Level &L = ctx->lv[level];
    const int nb = L.nb, Ne = ctx->mesh.Ne;
    if (L.inv_prec == FR_PREC_FP64)
        return (nb % 2 == 0) ? launch_apply<double, 2>(L, Ne, r, alpha, beta, yin, scale, y, s)
                             : launch_apply<double, 1>(L, Ne, r, alpha, beta, yin, scale, y, s);
    if (L.inv_prec == FR_PREC_BF16_STORE)
        return (nb % 4 == 0) ? launch_apply<__bf16, 4>(L, Ne, r, alpha, beta, yin, scale, y, s)
                             : launch_apply<__bf16, 1>(L, Ne, r, alpha, beta, yin, scale, y, s);
    if (L.inv_prec >= 0)
        return (nb % 4 == 0) ? launch_apply<float, 4>(L, Ne, r, alpha, beta, yin, scale, y, s)
                             : launch_apply<float, 1>(L, Ne, r, alpha, beta, yin, scale, y, s);
    return hipErrorInvalidValue;
}

hipError_t ej_apply(const frpmg_ctx *ctx, int level, const double *r, double alpha, double beta, double *y,
                    hipStream_t s) {
    return ej_apply_ex(ctx, level, r, alpha, beta, y, Scal{1.0, nullptr}, y, s);
}

}  // namespace frpmg
