// Vector kernels for the Krylov solver and the multigrid cycle (gfx950):
// dot products with a fixed two-pass reduction tree (run-to-run bitwise
// reproducible, no floating-point atomics), classical Gram-Schmidt
// multi-dots and updates, AXPBY-type updates with host or device scalars, and
// the p-multigrid restriction/prolongation.
#include "internal.hpp"

namespace frpmg {

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ double sget(const Scal &s) { return s.p ? *s.p : s.v; }

// 64-wide wavefront reduction, then across the 4 waves of the block.
__device__ __forceinline__ double block_sum(double v, double *s_red) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) s_red[wid] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) {
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) r += s_red[w];
    }
    __syncthreads();
    return r;
}

// partial[vec * nblk + block] = sum over this block's strided share of V_vec . w.
// The vectors are taken kChunk at a time with w read once per chunk; each
// vector's terms are still summed in the same order (so the result does not
// depend on the chunking).
constexpr int kChunk = 8;

__global__ void __launch_bounds__(kThreads) k_mdot_partial(size_t n, int nvec, const double *__restrict__ V,
                                                           size_t ldv, const double *__restrict__ w,
                                                           double *__restrict__ partial) {
    __shared__ double s_part[kChunk][kThreads / 64];
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    const size_t i0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int v0 = 0; v0 < nvec; v0 += kChunk) {
        const int nc = min(kChunk, nvec - v0);
        double acc[kChunk];
#pragma unroll
        for (int c = 0; c < kChunk; ++c) acc[c] = 0.0;
        for (size_t i = i0; i < n; i += stride) {
            const double wi = w[i];
#pragma unroll
            for (int c = 0; c < kChunk; ++c)
                if (c < nc) acc[c] += V[(size_t)(v0 + c) * ldv + i] * wi;
        }
        // the chunk's block sums in one pass: each wavefront reduces its nc
        // values by shuffles, then lane c of the block adds vector c's four
        // wavefront sums in wavefront order (the order of block_sum, so the
        // bits do not change), with one barrier per chunk instead of two per
        // vector
#pragma unroll
        for (int c = 0; c < kChunk; ++c) {
            if (c < nc) {
                double v = acc[c];
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
                if (lane == 0) s_part[c][wid] = v;
            }
        }
        __syncthreads();
        if ((int)threadIdx.x < nc) {
            double tot = 0.0;
            for (int w2 = 0; w2 < (int)(blockDim.x >> 6); ++w2) tot += s_part[threadIdx.x][w2];
            partial[(size_t)(v0 + threadIdx.x) * gridDim.x + blockIdx.x] = tot;
        }
        __syncthreads();  // s_part is rewritten by the next chunk
    }
}

// out[vec] = sum_b partial[vec * nblk + b], fixed order
__global__ void __launch_bounds__(kThreads) k_sum_partials(int nblk, const double *__restrict__ partial,
                                                           double *__restrict__ out) {
    __shared__ double s_red[kThreads / 64];
    const int vec = blockIdx.x;
    double acc = 0.0;
    for (int b = threadIdx.x; b < nblk; b += blockDim.x) acc += partial[(size_t)vec * nblk + b];
    const double tot = block_sum(acc, s_red);
    if (threadIdx.x == 0) out[vec] = tot;
}

// w -= sum_v h[v] V_v
__global__ void __launch_bounds__(kThreads) k_gemv_sub(size_t n, int nvec, const double *__restrict__ V,
                                                       size_t ldv, const double *__restrict__ h,
                                                       double *__restrict__ w) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        double acc = w[i];
        for (int vec = 0; vec < nvec; ++vec) acc -= h[vec] * V[(size_t)vec * ldv + i];
        w[i] = acc;
    }
}

// w -= sum_v h[v] V_v, then partial[vec * nblk + block] = this block's
// share of V_vec . w with the updated w: the update of one classical
// Gram-Schmidt pass and the products of the next in one pass over V (each
// lane keeps its NV entries of V in registers between the two).  The update
// takes the terms in k_gemv_sub's order and each product in
// k_mdot_partial's (same grid, same lane order, same reduction), so the
// results are bitwise those of the two kernels in turn.
constexpr int kFuseMax = 32;  // vectors per fused pass

template <int NV>
__global__ void __launch_bounds__(kThreads) k_gemv_sub_mdot(size_t n, const double *__restrict__ V, size_t ldv,
                                                            const double *__restrict__ h, double *__restrict__ w,
                                                            double *__restrict__ partial) {
    __shared__ double s_part[NV][kThreads / 64];
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    const size_t i0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    double hv[NV], acc[NV];
#pragma unroll
    for (int c = 0; c < NV; ++c) {
        hv[c] = h[c];
        acc[c] = 0.0;
    }
    for (size_t i = i0; i < n; i += stride) {
        double vv[NV];
#pragma unroll
        for (int c = 0; c < NV; ++c) vv[c] = V[(size_t)c * ldv + i];
        double wi = w[i];
#pragma unroll
        for (int c = 0; c < NV; ++c) wi -= hv[c] * vv[c];
        w[i] = wi;
#pragma unroll
        for (int c = 0; c < NV; ++c) acc[c] += vv[c] * wi;
    }
#pragma unroll
    for (int c = 0; c < NV; ++c) {
        double v = acc[c];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
        if (lane == 0) s_part[c][wid] = v;
    }
    __syncthreads();
    for (int c = threadIdx.x; c < NV; c += blockDim.x) {
        double tot = 0.0;
        for (int w2 = 0; w2 < (int)(blockDim.x >> 6); ++w2) tot += s_part[c][w2];
        partial[(size_t)c * gridDim.x + blockIdx.x] = tot;
    }
}

template <int NV>
void launch_gemv_sub_mdot(int nvec, unsigned nb, size_t n, const double *V, size_t ldv, const double *h, double *w,
                          double *partial, hipStream_t s) {
    if constexpr (NV <= kFuseMax) {
        if (nvec == NV)
            hipLaunchKernelGGL(k_gemv_sub_mdot<NV>, dim3(nb), dim3(kThreads), 0, s, n, V, ldv, h, w, partial);
        else
            launch_gemv_sub_mdot<NV + 1>(nvec, nb, n, V, ldv, h, w, partial, s);
    }
}

// y = y0 + sum_v c[v] Z_v  (y0 = y on entry)
__global__ void __launch_bounds__(kThreads) k_combine(size_t n, int nvec, const double *__restrict__ Z,
                                                      size_t ldz, const double *__restrict__ c,
                                                      double *__restrict__ y) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        double acc = y[i];
        for (int vec = 0; vec < nvec; ++vec) acc += c[vec] * Z[(size_t)vec * ldz + i];
        y[i] = acc;
    }
}

__global__ void __launch_bounds__(kThreads) k_axpby(size_t n, Scal a, const double *__restrict__ x, Scal b,
                                                    double *__restrict__ y) {
    const double av = sget(a), bv = sget(b);
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double yv = (bv == 0.0) ? 0.0 : bv * y[i];
        y[i] = (x ? av * x[i] : 0.0) + yv;
    }
}

__global__ void __launch_bounds__(kThreads) k_scale_copy(size_t n, Scal a, const double *__restrict__ x,
                                                         double *__restrict__ y) {
    const double av = sget(a);
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) y[i] = av * x[i];
}

// y = x / sqrt(n2): the reciprocal is formed as 1 / sqrt(n2), both correctly rounded
__global__ void __launch_bounds__(kThreads) k_normalize(size_t n, const double *__restrict__ n2,
                                                        const double *__restrict__ x, double *__restrict__ y) {
    const double av = 1.0 / sqrt(*n2);
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) y[i] = av * x[i];
}

__global__ void __launch_bounds__(kThreads) k_fill(size_t n, double v, double *__restrict__ y) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) y[i] = v;
}

__global__ void __launch_bounds__(kThreads) k_stage_F(size_t n, const double *__restrict__ x,
                                                      const double *__restrict__ b, double c,
                                                      const double *__restrict__ r, double *__restrict__ out) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        out[i] = (x[i] - b[i]) * c - r[i];
}

// Sum of the dot-product partials of one vector, in the order of
// k_sum_partials (so both give the same bits); every lane of block 0 calls it.
__device__ __forceinline__ double sum_partials_0(int nblk, const double *__restrict__ partial, double *s_red) {
    double acc = 0.0;
    for (int b = threadIdx.x; b < nblk; b += blockDim.x) acc += partial[b];
    return block_sum(acc, s_red);
}

// y = x / ||x|| with ||x||^2 summed from the partials by every block (same
// order as k_sum_partials, so every block sees the same bits); block 0
// also stores ||x||^2.
__global__ void __launch_bounds__(kThreads) k_sum_normalize(size_t n, int nblk, const double *__restrict__ partial,
                                                            double *n2out, const double *__restrict__ x,
                                                            double *__restrict__ y) {
    __shared__ double s_red[kThreads / 64];
    __shared__ double s_av;
    const double n2 = sum_partials_0(nblk, partial, s_red);
    if (threadIdx.x == 0) {
        if (blockIdx.x == 0) *n2out = n2;
        s_av = 1.0 / sqrt(n2);
    }
    __syncthreads();
    const double av = s_av;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) y[i] = av * x[i];
}

// ||v||^2 from the partials, then the FD step h = eps (1 + ||dq||) / ||v||
__global__ void __launch_bounds__(kThreads) k_sum_fd_step(int nblk, const double *__restrict__ partial,
                                                          const double *dqn2, double eps, double *n2out,
                                                          double *hout) {
    __shared__ double s_red[kThreads / 64];
    const double n2 = sum_partials_0(nblk, partial, s_red);
    if (threadIdx.x == 0) {
        *n2out = n2;
        const double size = dqn2 ? 1.0 + sqrt(*dqn2) : 1.0;
        *hout = (n2 > 0.0) ? eps * size / sqrt(n2) : eps;
    }
}

// ||X||^2 from the partials, then the preconditioner scale s and 1/s
__global__ void __launch_bounds__(kThreads) k_sum_pmg_scale(int nblk, const double *__restrict__ partial,
                                                            const double *qn2, double eps_p, double sigma,
                                                            double *n2out, double *s_out, double *inv_out) {
    __shared__ double s_red[kThreads / 64];
    const double n2 = sum_partials_0(nblk, partial, s_red);
    if (threadIdx.x == 0) {
        *n2out = n2;
        const double nrm = sqrt(n2);
        const double size = qn2 ? 1.0 + sqrt(*qn2) : 1.0;
        const double sc = (nrm > 0.0) ? eps_p * sigma * size / nrm : 1.0;
        *s_out = sc;
        *inv_out = 1.0 / sc;
    }
}

// h = eps (1 + ||dq||) / ||v||  (dqn2 = null: h = eps / ||v||)
__global__ void k_fd_step(const double *vn2, const double *dqn2, double eps, double *hout) {
    const double s = *vn2;
    const double size = dqn2 ? 1.0 + sqrt(*dqn2) : 1.0;
    *hout = (s > 0.0) ? eps * size / sqrt(s) : eps;
}

// s = eps_p sigma (1 + ||q||) / ||X||  (qn2 = null: without the state size)
__global__ void k_pmg_scale(const double *xn2, const double *qn2, double eps_p, double sigma, double *s_out,
                            double *inv_out) {
    const double nrm = sqrt(*xn2);
    const double size = qn2 ? 1.0 + sqrt(*qn2) : 1.0;
    const double s = (nrm > 0.0) ? eps_p * sigma * size / nrm : 1.0;
    *s_out = s;
    *inv_out = 1.0 / s;
}

unsigned grid_for(size_t n) {
    size_t b = (n + kThreads - 1) / kThreads;
    if (b > 4096) b = 4096;
    if (b == 0) b = 1;
    return (unsigned)b;
}

// partial sums per vector of a dot product of length n (fixed per n)
unsigned red_blocks(size_t n) {
    const unsigned nb = grid_for(n);
    const unsigned cap = n >= kRedLarge ? (unsigned)kRedBlocks : 512u;
    return nb > cap ? cap : nb;
}

// Restriction / prolongation with the 1D operator M (PO x PI) along each
// axis.  Sum-factorised: one lane per (variable, element) applies M along
// x, then y, then z, all in registers.  2D prolongation: one lane per (output
// point, element, variable) computes sum_j M[o1][j] sum_i M[o0][i] a[j][i]
// (the same operations in the same order as the sum-factorised form); 4096
// elements would otherwise give the chip only 64 workgroups, each lane
// writing PO^2 values (12.6 -> 8.0 us for p = 2 -> 4).  2D restriction keeps
// the sum-factorised form (it measured faster).  Compile-time sizes let
// the operator entries come from the kernel-argument segment with uniform
// indices.
struct Mat1D {
    double m[kMaxP][kMaxP];
};

// input x (minus x0 when given); output written, or added to y (acc).  With
// x2 given, lanes beyond the first vector map x2 to y2 (written, no x0).
template <int DIM, int PI, int PO>
__global__ void __launch_bounds__(kThreads) k_transfer_sf(int Ne, int nv, Mat1D M, const double *x1,
                                                          const double *x01, int acc1, double *y1,
                                                          const double *x2, double *y2) {
    constexpr int NI = (DIM == 2) ? PI * PI : PI * PI * PI;
    constexpr int NO = (DIM == 2) ? PO * PO : PO * PO * PO;
    constexpr int PZI = (DIM == 2) ? 1 : PI;
    constexpr int PZO = (DIM == 2) ? 1 : PO;
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const bool second = idx >= nv * Ne;
    if (second) {
        idx -= nv * Ne;
        if (!x2 || idx >= nv * Ne) return;
    }
    const double *__restrict__ x = second ? x2 : x1;
    const double *__restrict__ x0 = second ? nullptr : x01;
    const int acc = second ? 0 : acc1;
    double *__restrict__ y = second ? y2 : y1;
    const int k = idx % Ne, v = idx / Ne;
    double a[NI];
#pragma unroll
    for (int j = 0; j < NI; ++j) {
        const size_t i = ((size_t)v * NI + j) * Ne + k;
        a[j] = x0 ? x[i] - x0[i] : x[i];
    }
    double b[PZI * PI * PO];  // [z][y][x_out]
#pragma unroll
    for (int z = 0; z < PZI; ++z)
#pragma unroll
        for (int yy = 0; yy < PI; ++yy)
#pragma unroll
            for (int o = 0; o < PO; ++o) {
                double s = 0.0;
#pragma unroll
                for (int j = 0; j < PI; ++j) s += M.m[o][j] * a[(z * PI + yy) * PI + j];
                b[(z * PI + yy) * PO + o] = s;
            }
    double c[PZI * PO * PO];  // [z][y_out][x_out]
#pragma unroll
    for (int z = 0; z < PZI; ++z)
#pragma unroll
        for (int o1 = 0; o1 < PO; ++o1)
#pragma unroll
            for (int o0 = 0; o0 < PO; ++o0) {
                double s = 0.0;
#pragma unroll
                for (int j = 0; j < PI; ++j) s += M.m[o1][j] * b[(z * PI + j) * PO + o0];
                c[(z * PO + o1) * PO + o0] = s;
            }
    if (DIM == 2) {
#pragma unroll
        for (int o = 0; o < NO; ++o) {
            const size_t i = ((size_t)v * NO + o) * Ne + k;
            y[i] = acc ? y[i] + c[o] : c[o];
        }
    } else {
#pragma unroll
        for (int o2 = 0; o2 < PZO; ++o2)
#pragma unroll
            for (int o = 0; o < PO * PO; ++o) {
                double s = 0.0;
#pragma unroll
                for (int j = 0; j < PZI; ++j) s += M.m[o2][j] * c[j * PO * PO + o];
                const size_t i = ((size_t)v * NO + o2 * PO * PO + o) * Ne + k;
                y[i] = acc ? y[i] + s : s;
            }
    }
}

template <int PI, int PO>
__global__ void __launch_bounds__(kThreads) k_transfer_pt(int Ne, int nv, Mat1D M, const double *__restrict__ x,
                                                          const double *__restrict__ x0, int acc,
                                                          double *__restrict__ y) {
    constexpr int NI = PI * PI, NO = PO * PO;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nv * NO * Ne) return;
    const int k = idx % Ne, vo = idx / Ne;
    const int o = vo % NO, v = vo / NO;
    const int o1 = o / PO, o0 = o - o1 * PO;
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < PI; ++j) {
        double t = 0.0;
#pragma unroll
        for (int i = 0; i < PI; ++i) {
            const size_t ii = ((size_t)v * NI + j * PI + i) * Ne + k;
            t += M.m[o0][i] * (x0 ? x[ii] - x0[ii] : x[ii]);
        }
        s += M.m[o1][j] * t;
    }
    const size_t io = (size_t)idx;
    y[io] = acc ? y[io] + s : s;
}

template <int DIM, int PI, int PO>
void launch_sf(int Ne, int nv, const Mat1D &M, const double *x, const double *x0, int acc, double *y,
               const double *x2, double *y2, hipStream_t s) {
    if constexpr (DIM == 2 && PO > PI) {
        if (x2) launch_sf<DIM, PI, PO>(Ne, nv, M, x2, nullptr, 0, y2, nullptr, nullptr, s);
        const int n = nv * PO * PO * Ne;
        hipLaunchKernelGGL((k_transfer_pt<PI, PO>), dim3((n + kThreads - 1) / kThreads), dim3(kThreads), 0, s, Ne,
                           nv, M, x, x0, acc, y);
    } else {
        const int n = nv * Ne * (x2 ? 2 : 1);
        hipLaunchKernelGGL((k_transfer_sf<DIM, PI, PO>), dim3((n + kThreads - 1) / kThreads), dim3(kThreads), 0, s,
                           Ne, nv, M, x, x0, acc, y, x2, y2);
    }
}

template <int DIM>
bool dispatch_sf(int PI, int PO, int Ne, int nv, const Mat1D &M, const double *x, const double *x0, int acc,
                 double *y, const double *x2, double *y2, hipStream_t s) {
#define FR_SF(a, b) \
    if (PI == a && PO == b) { launch_sf<DIM, a, b>(Ne, nv, M, x, x0, acc, y, x2, y2, s); return true; }
    FR_SF(2, 3) FR_SF(2, 4) FR_SF(3, 2) FR_SF(3, 4) FR_SF(4, 2) FR_SF(4, 3) FR_SF(2, 1) FR_SF(1, 2)
    FR_SF(3, 1) FR_SF(1, 3) FR_SF(4, 1) FR_SF(1, 4)
    if (DIM == 2) {
        FR_SF(5, 2) FR_SF(2, 5) FR_SF(5, 3) FR_SF(3, 5) FR_SF(5, 4) FR_SF(4, 5) FR_SF(5, 1) FR_SF(1, 5)
    }
#undef FR_SF
    return false;
}

}  // namespace

hipError_t vec_dot(frpmg_ctx *ctx, size_t n, const double *x, const double *y, double *dout, hipStream_t s) {
    return vec_mdot(ctx, n, 1, x, 0, y, dout, s);
}

hipError_t vec_dot_fd_step(frpmg_ctx *ctx, size_t n, const double *v, const double *dqn2, double eps,
                           double *n2out, double *hout, hipStream_t s) {
    const unsigned nb = red_blocks(n);
    hipLaunchKernelGGL(k_mdot_partial, dim3(nb), dim3(kThreads), 0, s, n, 1, v, (size_t)0, v, ctx->red_partial);
    hipLaunchKernelGGL(k_sum_fd_step, dim3(1), dim3(kThreads), 0, s, (int)nb, ctx->red_partial, dqn2, eps, n2out,
                       hout);
    return hipGetLastError();
}

hipError_t vec_dot_normalize(frpmg_ctx *ctx, size_t n, const double *x, double *n2out, double *y, hipStream_t s) {
    const unsigned nb = red_blocks(n);
    hipLaunchKernelGGL(k_mdot_partial, dim3(nb), dim3(kThreads), 0, s, n, 1, x, (size_t)0, x, ctx->red_partial);
    hipLaunchKernelGGL(k_sum_normalize, dim3(grid_for(n)), dim3(kThreads), 0, s, n, (int)nb, ctx->red_partial, n2out,
                       x, y);
    return hipGetLastError();
}

hipError_t vec_dot_pmg_scale(frpmg_ctx *ctx, size_t n, const double *x, const double *qn2, double eps_p,
                             double sigma, double *n2out, double *s_out, double *inv_out, hipStream_t s) {
    const unsigned nb = red_blocks(n);
    hipLaunchKernelGGL(k_mdot_partial, dim3(nb), dim3(kThreads), 0, s, n, 1, x, (size_t)0, x, ctx->red_partial);
    hipLaunchKernelGGL(k_sum_pmg_scale, dim3(1), dim3(kThreads), 0, s, (int)nb, ctx->red_partial, qn2, eps_p, sigma,
                       n2out, s_out, inv_out);
    return hipGetLastError();
}

hipError_t vec_mdot(frpmg_ctx *ctx, size_t n, int nvec, const double *V, size_t ldv, const double *w,
                    double *dout, hipStream_t s) {
    const unsigned nb = red_blocks(n);
    hipLaunchKernelGGL(k_mdot_partial, dim3(nb), dim3(kThreads), 0, s, n, nvec, V, ldv, w, ctx->red_partial);
    hipLaunchKernelGGL(k_sum_partials, dim3(nvec), dim3(kThreads), 0, s, (int)nb, ctx->red_partial, dout);
    return hipGetLastError();
}

hipError_t vec_gemv_sub(size_t n, int nvec, const double *V, size_t ldv, const double *h, double *w,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_gemv_sub, dim3(grid_for(n)), dim3(kThreads), 0, s, n, nvec, V, ldv, h, w);
    return hipGetLastError();
}

hipError_t vec_gemv_sub_mdot(frpmg_ctx *ctx, size_t n, int nvec, const double *V, size_t ldv, const double *h,
                             double *w, double *dout, hipStream_t s) {
    if (nvec < 1 || nvec > kFuseMax) {
        hipError_t e = vec_gemv_sub(n, nvec, V, ldv, h, w, s);
        return e != hipSuccess ? e : vec_mdot(ctx, n, nvec, V, ldv, w, dout, s);
    }
    const unsigned nb = red_blocks(n);
    launch_gemv_sub_mdot<1>(nvec, nb, n, V, ldv, h, w, ctx->red_partial, s);
    hipLaunchKernelGGL(k_sum_partials, dim3(nvec), dim3(kThreads), 0, s, (int)nb, ctx->red_partial, dout);
    return hipGetLastError();
}

hipError_t vec_combine(size_t n, int nvec, const double *Z, size_t ldz, const double *c_dev, double *y,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_combine, dim3(grid_for(n)), dim3(kThreads), 0, s, n, nvec, Z, ldz, c_dev, y);
    return hipGetLastError();
}

hipError_t vec_axpby(size_t n, Scal a, const double *x, Scal b, double *y, hipStream_t s) {
    hipLaunchKernelGGL(k_axpby, dim3(grid_for(n)), dim3(kThreads), 0, s, n, a, x, b, y);
    return hipGetLastError();
}

hipError_t vec_normalize(size_t n, const double *n2, const double *x, double *y, hipStream_t s) {
    hipLaunchKernelGGL(k_normalize, dim3(grid_for(n)), dim3(kThreads), 0, s, n, n2, x, y);
    return hipGetLastError();
}

hipError_t vec_scale_copy(size_t n, Scal a, const double *x, double *y, hipStream_t s) {
    hipLaunchKernelGGL(k_scale_copy, dim3(grid_for(n)), dim3(kThreads), 0, s, n, a, x, y);
    return hipGetLastError();
}

hipError_t vec_fill(size_t n, double v, double *y, hipStream_t s) {
    hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(kThreads), 0, s, n, v, y);
    return hipGetLastError();
}

hipError_t vec_stage_F(size_t n, const double *x, const double *b, double c, const double *r, double *out,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_stage_F, dim3(grid_for(n)), dim3(kThreads), 0, s, n, x, b, c, r, out);
    return hipGetLastError();
}

hipError_t scal_fd_step(const double *vn2, const double *dqn2, double eps, double *hout, hipStream_t s) {
    hipLaunchKernelGGL(k_fd_step, dim3(1), dim3(1), 0, s, vn2, dqn2, eps, hout);
    return hipGetLastError();
}

hipError_t scal_pmg_scale(const double *xn2, const double *qn2, double eps_p, double sigma, double *s_out,
                          double *inv_out, hipStream_t s) {
    hipLaunchKernelGGL(k_pmg_scale, dim3(1), dim3(1), 0, s, xn2, qn2, eps_p, sigma, s_out, inv_out);
    return hipGetLastError();
}

namespace {

hipError_t transfer_launch(const frpmg_ctx *ctx, int fine_level, bool restrict_dir, const double *x, double *y,
                           const double *x0, bool accumulate, const double *x2, double *y2, hipStream_t s) {
    if (ctx->lv[fine_level].pa)
        return restrict_dir ? pa_transfer(ctx, fine_level, fine_level + 1, x, y, x0, accumulate, x2, y2, s)
                            : pa_transfer(ctx, fine_level + 1, fine_level, x, y, x0, accumulate, x2, y2, s);
    const Transfer1D &t = ctx->tr[fine_level];
    const int Pin = restrict_dir ? t.P0 : t.P1;
    const int Pout = restrict_dir ? t.P1 : t.P0;
    const int Ne = ctx->mesh.Ne;
    Mat1D M{};
    for (int o = 0; o < Pout; ++o)
        for (int j = 0; j < Pin; ++j) M.m[o][j] = restrict_dir ? t.G[o][j] : t.Pi[o][j];
    const int acc = accumulate ? 1 : 0;
    const bool ok = (ctx->dim == 2) ? dispatch_sf<2>(Pin, Pout, Ne, ctx->nv, M, x, x0, acc, y, x2, y2, s)
                                    : dispatch_sf<3>(Pin, Pout, Ne, ctx->nv, M, x, x0, acc, y, x2, y2, s);
    if (!ok) return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace

hipError_t transfer_apply(const frpmg_ctx *ctx, int fine_level, bool restrict_dir, const double *x, double *y,
                          hipStream_t s, const double *x0, bool accumulate) {
    return transfer_launch(ctx, fine_level, restrict_dir, x, y, x0, accumulate, nullptr, nullptr, s);
}

hipError_t transfer_restrict2(const frpmg_ctx *ctx, int fine_level, const double *x, double *y, const double *x2,
                              double *y2, hipStream_t s) {
    return transfer_launch(ctx, fine_level, true, x, y, nullptr, false, x2, y2, s);
}

}  // namespace frpmg
