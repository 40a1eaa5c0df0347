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

// partial[vec * nblk + block] = sum over this block's strided share of V_vec . w
__global__ void __launch_bounds__(kThreads) k_mdot_partial(size_t n, int nvec, const double *__restrict__ V,
                                                           size_t ldv, const double *__restrict__ w,
                                                           double *__restrict__ partial) {
    __shared__ double s_red[kThreads / 64];
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    const size_t i0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int vec = 0; vec < nvec; ++vec) {
        const double *x = V + (size_t)vec * ldv;
        double acc = 0.0;
        for (size_t i = i0; i < n; i += stride) acc += x[i] * w[i];
        const double tot = block_sum(acc, s_red);
        if (threadIdx.x == 0) partial[(size_t)vec * gridDim.x + blockIdx.x] = tot;
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

// Restriction / prolongation: y[v][i][k] = sum_j (M (x) M (x) M)[i][j] x[v][j][k]
// with the 1D operator M of the direction (tensor product over dim axes).
template <int DIM>
__global__ void __launch_bounds__(kThreads) k_transfer(int Ne, int Pin, int Pout, Transfer1D t, bool restr,
                                                       const double *__restrict__ x, double *__restrict__ y,
                                                       int nv) {
    const int Npo = (DIM == 2) ? Pout * Pout : Pout * Pout * Pout;
    const int Npi = (DIM == 2) ? Pin * Pin : Pin * Pin * Pin;
    const size_t total = (size_t)nv * Npo * Ne;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += stride) {
        const int k = (int)(idx % Ne);
        const size_t vi = idx / Ne;
        const int i = (int)(vi % Npo);
        const int v = (int)(vi / Npo);
        const int i0 = i % Pout, i1 = (i / Pout) % Pout, i2 = (DIM == 3) ? i / (Pout * Pout) : 0;
        double acc = 0.0;
        for (int j = 0; j < Npi; ++j) {
            const int j0 = j % Pin, j1 = (j / Pin) % Pin, j2 = (DIM == 3) ? j / (Pin * Pin) : 0;
            double w;
            if (restr) {
                w = t.G[i0][j0] * t.G[i1][j1];
                if (DIM == 3) w *= t.G[i2][j2];
            } else {
                w = t.Pi[i0][j0] * t.Pi[i1][j1];
                if (DIM == 3) w *= t.Pi[i2][j2];
            }
            acc += w * x[((size_t)v * Npi + j) * Ne + k];
        }
        y[idx] = acc;
    }
}

}  // namespace

hipError_t vec_dot(frpmg_ctx *ctx, size_t n, const double *x, const double *y, double *dout, hipStream_t s) {
    return vec_mdot(ctx, n, 1, x, 0, y, dout, s);
}

hipError_t vec_mdot(frpmg_ctx *ctx, size_t n, int nvec, const double *V, size_t ldv, const double *w,
                    double *dout, hipStream_t s) {
    unsigned nb = grid_for(n);
    if (nb > (unsigned)kRedBlocks) nb = kRedBlocks;
    hipLaunchKernelGGL(k_mdot_partial, dim3(nb), dim3(kThreads), 0, s, n, nvec, V, ldv, w, ctx->red_partial);
    hipLaunchKernelGGL(k_sum_partials, dim3(nvec), dim3(kThreads), 0, s, (int)nb, ctx->red_partial, dout);
    return hipGetLastError();
}

hipError_t vec_gemv_sub(size_t n, int nvec, const double *V, size_t ldv, const double *h, double *w,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_gemv_sub, dim3(grid_for(n)), dim3(kThreads), 0, s, n, nvec, V, ldv, h, w);
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

hipError_t transfer_apply(const frpmg_ctx *ctx, int fine_level, bool restrict_dir, const double *x, double *y,
                          hipStream_t s) {
    const Transfer1D &t = ctx->tr[fine_level];
    const int Pin = restrict_dir ? t.P0 : t.P1;
    const int Pout = restrict_dir ? t.P1 : t.P0;
    const int Ne = ctx->mesh.Ne;
    const size_t total = (size_t)ctx->nv * ctx->lv[restrict_dir ? fine_level + 1 : fine_level].Np * Ne;
    if (ctx->dim == 2)
        hipLaunchKernelGGL(k_transfer<2>, dim3(grid_for(total)), dim3(kThreads), 0, s, Ne, Pin, Pout, t,
                           restrict_dir, x, y, ctx->nv);
    else
        hipLaunchKernelGGL(k_transfer<3>, dim3(grid_for(total)), dim3(kThreads), 0, s, Ne, Pin, Pout, t,
                           restrict_dir, x, y, ctx->nv);
    return hipGetLastError();
}

}  // namespace frpmg
