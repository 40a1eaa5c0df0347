// Element-Jacobi blocks on gfx950: inversion of every block (Sec. 2.2,
// element-Jacobi preconditioner; Sec. 3.2, EJ smoother).  The batched apply
// with the stored inverses is in ej_apply.hip.
//
// Inversion: one workgroup per block, the whole FP64 block resident in LDS
// (n_b <= 140 fits in the 160 KB of a CU), Gauss-Jordan elimination with
// partial pivoting (largest |a|, first row on ties), the inverse written
// back column-major in the requested storage precision.  Larger blocks, and
// the BF16-MFMA precision form at any size, use the blocked variant below.  Storing the inverse
// turns every apply into a batched GEMV that streams the blocks once from
// HBM with coalesced column reads, with no sequential triangular sweeps.
#include <utility>

#include "internal.hpp"

namespace frpmg {

namespace {

constexpr int kGJThreads = 256;
constexpr int kMaxLdsBlock = 140;

__device__ __forceinline__ void argmax_combine(double &v, int &i, double v2, int i2) {
    if (v2 > v || (v2 == v && i2 < i)) {
        v = v2;
        i = i2;
    }
}

template <typename T>
__global__ void __launch_bounds__(kGJThreads) k_gj_invert(int nb, const double *__restrict__ B, T *__restrict__ out,
                                                          int *__restrict__ status) {
    extern __shared__ double A[];  // nb * nb, column-major: A[col * nb + row]
    double *colk = A + (size_t)nb * nb;
    __shared__ int perm[kMaxLdsBlock];
    __shared__ double s_v[kGJThreads / 64];
    __shared__ int s_i[kGJThreads / 64];
    __shared__ int s_piv;
    const int tid = threadIdx.x, nt = blockDim.x;
    const size_t base = (size_t)blockIdx.x * nb * nb;
    // elimination layout: lane = (row er, column group eg), rows padded to a
    // multiple of 64 so that a wave never straddles two column groups
    const int RT = min(nt, ((nb + 63) / 64) * 64);
    const int er = tid % RT, eg = tid / RT, ng = nt / RT;
    for (int t = tid; t < nb * nb; t += nt) A[t] = B[base + t];
    __syncthreads();
    bool singular = false;
    for (int c = 0; c < nb; ++c) {
        // pivot search in column c, rows c..nb-1
        double best = -1.0;
        int bi = 0x7fffffff;
        for (int r = c + tid; r < nb; r += nt) argmax_combine(best, bi, fabs(A[c * nb + r]), r);
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const double v2 = __shfl_down(best, off, 64);
            const int i2 = __shfl_down(bi, off, 64);
            argmax_combine(best, bi, v2, i2);
        }
        if ((tid & 63) == 0) {
            s_v[tid >> 6] = best;
            s_i[tid >> 6] = bi;
        }
        __syncthreads();
        if (tid == 0) {
            double bv = s_v[0];
            int ii = s_i[0];
            for (int w = 1; w < nt / 64; ++w) argmax_combine(bv, ii, s_v[w], s_i[w]);
            s_piv = ii;
            perm[c] = ii;
        }
        __syncthreads();
        const int p = s_piv;
        if (p != c) {
            for (int j = tid; j < nb; j += nt) {
                const double t0 = A[j * nb + c];
                A[j * nb + c] = A[j * nb + p];
                A[j * nb + p] = t0;
            }
        }
        __syncthreads();
        double d = A[c * nb + c];
        if (d == 0.0) {
            singular = true;
            d = 1.0;
        }
        const double inv = 1.0 / d;
        for (int r = tid; r < nb; r += nt) colk[r] = A[c * nb + r];
        __syncthreads();
        for (int j = tid; j < nb; j += nt) A[j * nb + c] = (j == c ? 1.0 : A[j * nb + c]) * inv;
        __syncthreads();
        if (er < nb && er != c && eg < ng) {
            // rows other than c never write the pivot row, so the pivot-row
            // reads of four columns can be issued ahead of the updates
            const double f = colk[er];
            int j = eg;
            for (; j + 3 * ng < nb; j += 4 * ng) {
                double a[4], pv[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    a[u] = A[(j + u * ng) * nb + er];
                    pv[u] = A[(j + u * ng) * nb + c];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const double cur = (j + u * ng == c) ? 0.0 : a[u];
                    A[(j + u * ng) * nb + er] = cur - f * pv[u];
                }
            }
            for (; j < nb; j += ng) {
                const double cur = (j == c) ? 0.0 : A[j * nb + er];
                A[j * nb + er] = cur - f * A[j * nb + c];
            }
        }
        __syncthreads();
    }
    // undo the row interchanges as column interchanges, last first
    for (int c = nb - 1; c >= 0; --c) {
        const int p = perm[c];
        if (p != c) {
            for (int r = tid; r < nb; r += nt) {
                const double t0 = A[c * nb + r];
                A[c * nb + r] = A[p * nb + r];
                A[p * nb + r] = t0;
            }
        }
        __syncthreads();
    }
    for (int t = tid; t < nb * nb; t += nt) out[base + t] = (T)A[t];
    if (singular && tid == 0) status[0] = 1;
}

// ---------------------------------------------------------------------------
// Blocked in-place Gauss-Jordan for blocks too large for LDS (n_b > 140, e.g.
// 320 x 320 in 3D at p = 3).  Panels of kPanel columns are eliminated in registers
// (pivot search over the full column, row swaps recorded); the product of the
// panel's elementary transforms T = (I + W S^T) P (S = the panel's pivot rows)
// is then applied to every other column at once as a GEMM:
//     x <- (P x with the pivot rows zeroed) + T_panel (P x)_S,
// where T_panel = the panel columns just written back.  After the last panel
// the row interchanges are undone as column interchanges, last first.
// ---------------------------------------------------------------------------
constexpr int kPanel = 32;

// Panel factorisation with the panel in registers: lane r owns row r of the
// panel (kPanel values).  Per pivot step: the argmax of |column| over rows
// >= c (wavefront shuffles, then across wavefronts through LDS; the lowest
// row wins ties), then the pivot row and row c are exchanged through LDS,
// every lane reads the pivot row and updates its own row.  Three barriers per
// step and under 1 KB of LDS, so several blocks share a CU.  The steps are
// instantiated per panel column so that every register index is a constant
// (a runtime index would put the row in scratch memory).
struct PanelLds {
    double v[8];
    int i[8];
    int piv;
    double pivrow[kPanel];  // the pivot row (old row p)
    double oldc[kPanel];    // old row c, taken over by lane p
};

template <int CC>
__device__ __forceinline__ void panel_step(double (&x)[kPanel], PanelLds &sh, int r, int nb, int c0, int bw,
                                           int nw, int *__restrict__ perm, bool &singular) {
    if (CC >= bw) return;
    const int c = c0 + CC;
    double best = (r >= c && r < nb) ? fabs(x[CC]) : -1.0;
    int bi = (r >= c && r < nb) ? r : 0x7fffffff;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const double v2 = __shfl_down(best, off, 64);
        const int i2 = __shfl_down(bi, off, 64);
        argmax_combine(best, bi, v2, i2);
    }
    if ((r & 63) == 0) {
        sh.v[r >> 6] = best;
        sh.i[r >> 6] = bi;
    }
    __syncthreads();
    if (r == 0) {
        double bv = sh.v[0];
        int ii = sh.i[0];
        for (int w = 1; w < nw; ++w) argmax_combine(bv, ii, sh.v[w], sh.i[w]);
        sh.piv = ii;
        perm[(size_t)blockIdx.x * nb + c] = ii;
    }
    __syncthreads();
    const int p = sh.piv;
    if (r == p) {
#pragma unroll
        for (int j = 0; j < kPanel; ++j) sh.pivrow[j] = x[j];
    }
    if (r == c && p != c) {
#pragma unroll
        for (int j = 0; j < kPanel; ++j) sh.oldc[j] = x[j];
    }
    __syncthreads();
    if (r == p && p != c) {
#pragma unroll
        for (int j = 0; j < kPanel; ++j) x[j] = sh.oldc[j];
    }
    double d = sh.pivrow[CC];
    if (d == 0.0) {
        singular = true;
        d = 1.0;
    }
    const double inv = 1.0 / d;
    if (r == c) {
#pragma unroll
        for (int j = 0; j < kPanel; ++j) x[j] = (j == CC ? 1.0 : sh.pivrow[j]) * inv;
    } else if (r < nb) {
        const double f = x[CC];
#pragma unroll
        for (int j = 0; j < kPanel; ++j) {
            const double pv = (j == CC ? 1.0 : sh.pivrow[j]) * inv;
            x[j] = (j == CC ? 0.0 : x[j]) - f * pv;
        }
    }
}

template <int... CC>
__device__ __forceinline__ void panel_steps(std::integer_sequence<int, CC...>, double (&x)[kPanel], PanelLds &sh,
                                            int r, int nb, int c0, int bw, int nw, int *__restrict__ perm,
                                            bool &singular) {
    (panel_step<CC>(x, sh, r, nb, c0, bw, nw, perm, singular), ...);
}

__global__ void __launch_bounds__(512) k_gj_panel_reg(int nb, int c0, int bw, double *__restrict__ A,
                                                      int *__restrict__ perm, int *__restrict__ status) {
    __shared__ PanelLds sh;
    const int r = threadIdx.x;
    const int nw = blockDim.x >> 6;
    double *Ak = A + (size_t)blockIdx.x * nb * nb;
    double x[kPanel];
#pragma unroll
    for (int j = 0; j < kPanel; ++j) x[j] = (r < nb && j < bw) ? Ak[(size_t)(c0 + j) * nb + r] : 0.0;
    bool singular = false;
    panel_steps(std::make_integer_sequence<int, kPanel>{}, x, sh, r, nb, c0, bw, nw, perm, singular);
    if (r < nb) {
#pragma unroll
        for (int j = 0; j < kPanel; ++j)
            if (j < bw) Ak[(size_t)(c0 + j) * nb + r] = x[j];
    }
    if (singular && r == 0) status[0] = 1;
}

constexpr int kUpdCols = 64;  // columns per update workgroup
constexpr int kUpdRows = 64;  // rows per LDS chunk of T_panel
constexpr int kMaxNb = 512;   // largest block the update kernels take

// The row interchanges of one panel, applied by gathering instead of swapping
// in place.  LDS state of one workgroup: src[r] = the row whose value ends at
// row r after the panel's interchanges (identity outside the touched rows),
// upos[r] = index of row r in the list of touched rows U (-1 if untouched),
// and stage[u][jj] = the old value at touched row U[u] of tile column jj.
struct PanelPerm {
    int src[kMaxNb];
    int upos[kMaxNb];
    int rows[2 * kPanel];
    int nu;
};

// Fill a PanelPerm for block k (all lanes take part; ends with a barrier).
__device__ __forceinline__ void panel_perm(PanelPerm &pp, int nb, int c0, int bw, const int *__restrict__ perm,
                                           int k) {
    for (int r = threadIdx.x; r < nb; r += blockDim.x) {
        pp.src[r] = r;
        pp.upos[r] = -1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int nu = 0;
        for (int cc = 0; cc < bw; ++cc) {
            const int c = c0 + cc, p = perm[(size_t)k * nb + c];
            const int t = pp.src[c];
            pp.src[c] = pp.src[p];
            pp.src[p] = t;
            if (pp.upos[c] < 0) {
                pp.upos[c] = nu;
                pp.rows[nu++] = c;
            }
            if (pp.upos[p] < 0) {
                pp.upos[p] = nu;
                pp.rows[nu++] = p;
            }
        }
        pp.nu = nu;
    }
    __syncthreads();
}

// stage[u][jj] = old value of touched row U[u] in tile column jj (0 beyond
// the block's columns); every lane takes part, ends with a barrier.
__device__ __forceinline__ void stage_touched(const PanelPerm &pp, double (*stage)[kUpdCols], const double *Ak,
                                              int nb, int c0, int bw, int tile) {
    const int nrest = nb - bw;
    for (int t = threadIdx.x; t < pp.nu * kUpdCols; t += blockDim.x) {
        const int u = t / kUpdCols, jj = t % kUpdCols;
        const int ri = tile * kUpdCols + jj;
        double v = 0.0;
        if (ri < nrest) {
            const int j = (ri < c0) ? ri : ri + bw;
            v = Ak[(size_t)j * nb + pp.rows[u]];
        }
        stage[u][jj] = v;
    }
    __syncthreads();
}

// (P x)[r] of tile column jj: from the stage for touched rows, else from x
__device__ __forceinline__ double permuted(const PanelPerm &pp, const double (*stage)[kUpdCols], const double *x,
                                           int r, int jj) {
    return pp.upos[r] >= 0 ? stage[pp.upos[pp.src[r]]][jj] : x[r];
}

// Apply the panel transform to the kUpdCols columns (outside the panel) of
// one block: 256 lanes, each owns a 4 x 4 register tile of the output chunk.
__global__ void __launch_bounds__(256) k_gj_update(int nb, int c0, int bw, double *__restrict__ A,
                                                   const int *__restrict__ perm) {
    __shared__ double xs[kPanel][kUpdCols];    // (P x)_S for the tile's columns
    __shared__ double tp[kPanel][kUpdRows];    // T_panel rows chunk
    const int tid = threadIdx.x;
    const int k = blockIdx.x;
    double *Ak = A + (size_t)k * nb * nb;
    const int nrest = nb - bw;
    const int ri = blockIdx.y * kUpdCols + (tid % kUpdCols);  // rest-column index of this lane (phase 1)
    // phase 1: row interchanges on the tile's columns in place (32 KB of LDS
    // keeps five workgroups per CU, which beats the gather of the MFMA variant
    // here), then gather (P x)_S
    if (tid < kUpdCols) {
        if (ri < nrest) {
            const int j = (ri < c0) ? ri : ri + bw;
            double *x = Ak + (size_t)j * nb;
            for (int cc = 0; cc < bw; ++cc) {
                const int c = c0 + cc, p = perm[(size_t)k * nb + c];
                if (p != c) {
                    const double t0 = x[c];
                    x[c] = x[p];
                    x[p] = t0;
                }
            }
            for (int cc = 0; cc < bw; ++cc) xs[cc][tid] = x[c0 + cc];
        } else {
            for (int cc = 0; cc < bw; ++cc) xs[cc][tid] = 0.0;
        }
    }
    __syncthreads();
    // phase 2: out[r][j] = (r in S ? 0 : x[r]) + sum_cc T[r][cc] xs[cc][j]
    const int tr = (tid % 16) * 4;  // 4 rows
    const int tc = (tid / 16) * 4;  // 4 columns
    for (int r0 = 0; r0 < nb; r0 += kUpdRows) {
        for (int t = tid; t < bw * kUpdRows; t += 256) {
            const int cc = t / kUpdRows, rr = t % kUpdRows;
            tp[cc][rr] = (r0 + rr < nb) ? Ak[(size_t)(c0 + cc) * nb + r0 + rr] : 0.0;
        }
        __syncthreads();
        double acc[4][4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
        for (int cc = 0; cc < bw; ++cc) {
            double tv[4], xv[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) tv[a] = tp[cc][tr + a];
#pragma unroll
            for (int b = 0; b < 4; ++b) xv[b] = xs[cc][tc + b];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) acc[a][b] += tv[a] * xv[b];
        }
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int rib = blockIdx.y * kUpdCols + tc + b;
            if (rib >= nrest) continue;
            const int j = (rib < c0) ? rib : rib + bw;
            double *x = Ak + (size_t)j * nb;
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                const int r = r0 + tr + a;
                if (r >= nb) continue;
                const bool inS = (r >= c0 && r < c0 + bw);
                x[r] = (inS ? 0.0 : x[r]) + acc[a][b];
            }
        }
        __syncthreads();
    }
}

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

// The same panel update on BF16-input MFMA with FP32 accumulation
// (v_mfma_f32_16x16x32_bf16, K = the 32-column panel): each FP32 operand is
// split into hi + lo BF16 parts and the product taken as hi*hi + hi*lo +
// lo*hi (three MFMAs), ~16 mantissa bits.  Operands are staged k-contiguous
// in LDS; wave w owns 16 output rows of the 64-row chunk and the four 16-column
// blocks of the workgroup's 64 columns.
__global__ void __launch_bounds__(256) k_gj_update_mfma(int nb, int c0, int bw, double *__restrict__ A,
                                                        const int *__restrict__ perm) {
    __shared__ __attribute__((aligned(16))) __bf16 xs_h[kUpdCols][kPanel];
    __shared__ __attribute__((aligned(16))) __bf16 xs_l[kUpdCols][kPanel];
    __shared__ __attribute__((aligned(16))) __bf16 tp_h[kUpdRows][kPanel];
    __shared__ __attribute__((aligned(16))) __bf16 tp_l[kUpdRows][kPanel];
    __shared__ double stage[2 * kPanel][kUpdCols];
    __shared__ PanelPerm pp;
    const int tid = threadIdx.x;
    const int k = blockIdx.x;
    double *Ak = A + (size_t)k * nb * nb;
    const int nrest = nb - bw;
    // phase 1: the panel's row interchanges as a gather, (P x)_S split in hi/lo
    panel_perm(pp, nb, c0, bw, perm, k);
    stage_touched(pp, stage, Ak, nb, c0, bw, blockIdx.y);
    for (int t = tid; t < kPanel * kUpdCols; t += 256) {
        const int cc = t % kPanel, jj = t / kPanel;
        const float v = (cc < bw) ? (float)stage[pp.upos[pp.src[c0 + cc]]][jj] : 0.f;
        const __bf16 h = (__bf16)v;
        xs_h[jj][cc] = h;
        xs_l[jj][cc] = (__bf16)(v - (float)h);
    }
    __syncthreads();
    const int lane = tid & 63, wave = tid >> 6;
    const int r16 = lane & 15, g = lane >> 4;
    for (int r0 = 0; r0 < nb; r0 += kUpdRows) {
        for (int t = tid; t < kPanel * kUpdRows; t += 256) {
            const int cc = t / kUpdRows, rr = t % kUpdRows;
            const float v = (cc < bw && r0 + rr < nb) ? (float)Ak[(size_t)(c0 + cc) * nb + r0 + rr] : 0.f;
            const __bf16 h = (__bf16)v;
            tp_h[rr][cc] = h;
            tp_l[rr][cc] = (__bf16)(v - (float)h);
        }
        __syncthreads();
        const int arow = wave * 16 + r16;
        const bf16x8_t ah = *reinterpret_cast<const bf16x8_t *>(&tp_h[arow][8 * g]);
        const bf16x8_t al = *reinterpret_cast<const bf16x8_t *>(&tp_l[arow][8 * g]);
#pragma unroll
        for (int cb = 0; cb < kUpdCols / 16; ++cb) {
            const int bcol = cb * 16 + r16;
            const bf16x8_t bh = *reinterpret_cast<const bf16x8_t *>(&xs_h[bcol][8 * g]);
            const bf16x8_t bl = *reinterpret_cast<const bf16x8_t *>(&xs_l[bcol][8 * g]);
            f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc, 0, 0, 0);
            const int rib = blockIdx.y * kUpdCols + bcol;
            if (rib < nrest) {
                const int j = (rib < c0) ? rib : rib + bw;
                double *x = Ak + (size_t)j * nb;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int r = r0 + wave * 16 + 4 * g + i;
                    if (r >= nb) continue;
                    const bool inS = (r >= c0 && r < c0 + bw);
                    x[r] = (inS ? 0.0 : permuted(pp, stage, x, r, bcol)) + (double)acc[i];
                }
            }
        }
        __syncthreads();
    }
}

// Undo the row interchanges as column interchanges, last first.
__global__ void __launch_bounds__(256) k_gj_unscramble(int nb, double *__restrict__ A, const int *__restrict__ perm) {
    double *Ak = A + (size_t)blockIdx.x * nb * nb;
    for (int c = nb - 1; c >= 0; --c) {
        const int p = perm[(size_t)blockIdx.x * nb + c];
        if (p != c) {
            for (int r = threadIdx.x; r < nb; r += blockDim.x) {
                const double t0 = Ak[(size_t)c * nb + r];
                Ak[(size_t)c * nb + r] = Ak[(size_t)p * nb + r];
                Ak[(size_t)p * nb + r] = t0;
            }
        }
        __syncthreads();
    }
}

__global__ void k_to_float(size_t n, const double *__restrict__ a, float *__restrict__ b) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) b[i] = (float)a[i];
}

__global__ void k_to_bf16(size_t n, const double *__restrict__ a, __bf16 *__restrict__ b) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) b[i] = (__bf16)(float)a[i];
}

}  // namespace

hipError_t ej_invert(frpmg_ctx *ctx, int level, int precision, hipStream_t s) {
    Level &L = ctx->lv[level];
    const int nb = L.nb, Ne = ctx->mesh.Ne;
    if (nb > kMaxLdsBlock || precision == FR_PREC_FP32_BF16 || precision == FR_PREC_BF16_STORE) {
        if (nb > 512 || !L.perm) return hipErrorInvalidValue;
        const bool mfma = precision != FR_PREC_FP64;
        const int rows = ((nb + 63) / 64) * 64;  // one lane per block row
        for (int c0 = 0; c0 < nb; c0 += kPanel) {
            const int bw = min(kPanel, nb - c0);
            hipLaunchKernelGGL(k_gj_panel_reg, dim3(Ne), dim3(rows), 0, s, nb, c0, bw, L.blk64, L.perm, L.dstatus);
            const int nrest = nb - bw;
            if (nrest > 0) {
                const dim3 gu(Ne, (nrest + kUpdCols - 1) / kUpdCols);
                if (mfma)
                    hipLaunchKernelGGL(k_gj_update_mfma, gu, dim3(256), 0, s, nb, c0, bw, L.blk64, L.perm);
                else
                    hipLaunchKernelGGL(k_gj_update, gu, dim3(256), 0, s, nb, c0, bw, L.blk64, L.perm);
            }
        }
        hipLaunchKernelGGL(k_gj_unscramble, dim3(Ne), dim3(256), 0, s, nb, L.blk64, L.perm);
        const size_t n = (size_t)Ne * nb * nb;
        if (precision == FR_PREC_FP64) {
            L.inv = L.blk64;
        } else if (precision == FR_PREC_BF16_STORE) {
            hipLaunchKernelGGL(k_to_bf16, dim3(4096), dim3(256), 0, s, n, L.blk64, L.inv16);
            L.inv = L.inv16;
        } else {
            hipLaunchKernelGGL(k_to_float, dim3(4096), dim3(256), 0, s, n, L.blk64, L.inv32);
            L.inv = L.inv32;
        }
        L.inv_prec = precision;
        return hipGetLastError();
    }
    const size_t lds = ((size_t)nb * nb + nb) * sizeof(double);
    hipError_t e;
    if (precision == FR_PREC_FP64) {
        e = hipFuncSetAttribute((const void *)k_gj_invert<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_gj_invert<double>, dim3(Ne), dim3(kGJThreads), lds, s, nb, L.blk64, L.blk64,
                           L.dstatus);
        L.inv = L.blk64;
    } else {
        e = hipFuncSetAttribute((const void *)k_gj_invert<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_gj_invert<float>, dim3(Ne), dim3(kGJThreads), lds, s, nb, L.blk64, L.inv32,
                           L.dstatus);
        L.inv = L.inv32;
    }
    L.inv_prec = precision;
    return hipGetLastError();
}

}  // namespace frpmg
