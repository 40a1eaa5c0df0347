// Matrix-based Newton-Krylov (MBNK) smoother on gfx950 (Sec. 3.2): the
// coarsest pMG level solves its linearised pseudo-time step
//   (sigma I - dR/dq) delta = G
// by GMRES with at most five iterations to a relative tolerance of 1e-1,
// right-preconditioned by ILU0, instead of one element-Jacobi application.
//
// The assembled operator keeps, for every element k, the diagonal block and
// the 2 dim blocks that couple k to its face neighbours.  The off-diagonal
// blocks come from one-sided differences of the residual, many elements
// perturbed at once: elements of one colour lie at least three apart along
// some axis, so the residual stencils of two perturbed elements (the element
// and its face and edge neighbours) are disjoint and every difference
// belongs to one perturbation.  A 2D level evaluates many (colour, column)
// perturbations in one batched residual launch, each copy of the mesh being
// an independent slab of elements.
//
// ILU0 runs in red-black element order.  With face couplings only, red rows
// have no lower part, so the factorisation keeps D_r for red elements and
// the Schur complements U_b = D_b - sum_r O_br D_r^{-1} O_rb for black ones
// (ILU0 drops the fill between distinct black elements), and both
// triangular solves are three element-parallel steps.  Every decision of the
// GMRES cycle (convergence, breakdown) is taken on the device, so a sweep is
// a fixed sequence of launches that a HIP graph can capture.
#include "internal.hpp"

namespace frpmg {

namespace {

constexpr int kThreads = 256;

// device scalars of one GMRES cycle (doubles)
constexpr int GM_H1 = 0;       // first Gram-Schmidt pass, up to 8 values
constexpr int GM_H2 = 8;       // second pass
constexpr int GM_N2 = 16;      // squared norm of the last normalised vector
constexpr int GM_TARGET = 17;  // tol ||G||
constexpr int GM_DONE = 18;    // 1 once the cycle has stopped
constexpr int GM_JEND = 19;    // iterations whose directions form the update
constexpr int GM_G = 24;       // rotated right-hand side, 9 values
constexpr int GM_CS = 33;      // rotations, 8 each
constexpr int GM_SN = 41;
constexpr int GM_Y = 49;       // least-squares solution, 8 values
constexpr int GM_H = 64;       // Hessenberg matrix, column-major 9 x 8
constexpr int GM_SIZE = 64 + 9 * 8;
constexpr int kMaxIt = kMbnkMaxIt;

// the element of colour col (0 red, 1 black) among elements 2c and 2c + 1
// (an even element count along axis 0 keeps both in one row)
__device__ __forceinline__ int colour_elem(const MeshK &m, int c, int col) {
    int x[3];
    const int k0 = 2 * c;
    coords(m, k0, x);
    const int par = (x[0] + x[1] + (m.dim == 3 ? x[2] : 0)) & 1;
    return par == col ? k0 : k0 + 1;
}

// colour of the neighbour-block differences: sum_a (c_a mod s_a) prod_{b<a} s_b
__device__ __forceinline__ int fd_colour(const MeshK &m, int s0, int s1, int s2, int k) {
    int x[3];
    coords(m, k, x);
    int col = x[0] % s0 + s0 * (x[1] % s1);
    if (m.dim == 3) col += s0 * s1 * (x[2] % s2);
    return col;
}

// qb[vi][b][k] = dq[vi][k], plus the step where pair p0 + b perturbs (vi, k)
__global__ void __launch_bounds__(kThreads) k_mb_perturb(MeshK m, int nb, int Np, Phys ph, int s0, int s1, int s2,
                                                         int p0, int cnt, const double *__restrict__ dq,
                                                         double *__restrict__ qb) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m.Ne) return;
    const int row = blockIdx.y;  // vi cnt + b
    const int vi = row / cnt, b = row - vi * cnt;
    const int pair = p0 + b;
    const int colour = pair / nb, j = pair - colour * nb;
    double u = dq[(size_t)vi * m.Ne + k];
    if (vi == j && fd_colour(m, s0, s1, s2, k) == colour) u = u + fd_step(ph.qinf[vi / Np], u);
    qb[((size_t)vi * cnt + b) * m.Ne + k] = u;
}

// O[k][slot(a, -side)][:, j] = -(R_b[:, k] - r0[:, k]) / h_m for every member
// m of the pair's colour and k its face neighbour (a, side)
__global__ void __launch_bounds__(kThreads) k_mb_extract(MeshK m, int nb, int Np, Phys ph, int s0, int s1, int s2,
                                                         int p0, int cnt, int nface, const double *__restrict__ dq,
                                                         const double *__restrict__ r0,
                                                         const double *__restrict__ rb, double *__restrict__ O) {
    const int b = blockIdx.y / nface, f = blockIdx.y - b * nface;
    const int pair = p0 + b;
    const int colour = pair / nb, j = pair - colour * nb;
    const int M0 = m.n[0] / s0, M1 = m.n[1] / s1, M2 = (m.dim == 3) ? m.n[2] / s2 : 1;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= M0 * M1 * M2 * nb) return;
    const int mu = t / nb, row = t - mu * nb;
    int c[3];
    c[0] = colour % s0 + s0 * (mu % M0);
    c[1] = (colour / s0) % s1 + s1 * ((mu / M0) % M1);
    c[2] = (m.dim == 3) ? (colour / (s0 * s1)) + s2 * (mu / (M0 * M1)) : 0;
    const int mel = elem_index(m, c);
    const int k = neighbour(m, mel, f >> 1, (f & 1) ? 1 : -1);
    const double base = dq[(size_t)j * m.Ne + mel];
    const double h = (base + fd_step(ph.qinf[j / Np], base)) - base;
    const double Rk = rb[((size_t)row * cnt + b) * m.Ne + k];
    O[((size_t)k * nface + (f ^ 1)) * nb * nb + (size_t)j * nb + row] = -(Rk - r0[(size_t)row * m.Ne + k]) / h;
}

__global__ void __launch_bounds__(kThreads) k_mb_gather(MeshK m, int nb, int col, const double *__restrict__ D,
                                                        double *__restrict__ out) {
    const int c = blockIdx.x;
    const int k = colour_elem(m, c, col);
    const size_t nn = (size_t)nb * nb;
    for (size_t t = threadIdx.x; t < nn; t += blockDim.x) out[c * nn + t] = D[(size_t)k * nn + t];
}

// One nb x nb block (column-major) read through a buffer resource: a read
// outside the block (row or column >= nb, the padding of the 16 x 16 tiles)
// returns 0 from the range check, so the operand loads carry no branches.
typedef double f64x4_t __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));
struct BlockRd {
    __amdgpu_buffer_rsrc_t rs;
    int nb;
    __device__ BlockRd(const double *p, int nb_)
        : rs(__builtin_amdgcn_make_buffer_rsrc(const_cast<double *>(p), (short)0, nb_ * nb_ * (int)sizeof(double),
                                               0x00020000)),
          nb(nb_) {}
    __device__ __forceinline__ double at(int i, int j) const {
        const unsigned off = (i < nb && j < nb) ? (unsigned)(j * nb + i) * (unsigned)sizeof(double) : 0x80000000u;
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0));
    }
};

// acc[q] += A[16 it + rows][k] B[k][16 (jt0 + q) + cols] over k < nb on
// v_mfma_f64_16x16x4f64 (lane (r16, g): A row r16, k = 4 ks + g; B k = 4 ks +
// g, column r16; result rows g + 4v, column r16), for nq <= 3 column tiles.
// The operands of the next four k steps are read while the current four
// are multiplied.
template <typename LA, typename LB>
__device__ __forceinline__ void schur_tiles(int nb, int it, int jt0, int nq, const LA &la, const LB &lb,
                                            f64x4_t (&acc)[3]) {
    const int lane = threadIdx.x & 63, r16 = lane & 15, g = lane >> 4;
    const int i = it * 16 + r16;
    int jc[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) jc[q] = (jt0 + (q < nq ? q : 0)) * 16 + r16;
    double a[2][4], bb[2][4][3];
    auto load = [&](int buf, int k0) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int k = k0 + 4 * u + g;
            a[buf][u] = la(i, k);
#pragma unroll
            for (int q = 0; q < 3; ++q) bb[buf][u][q] = lb(k, jc[q]);
        }
    };
    auto mma = [&](int buf) {
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int q = 0; q < 3; ++q)
                if (q < nq) acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[buf][u], bb[buf][u][q], acc[q], 0, 0, 0);
    };
    const int nk = (nb + 15) / 16;  // blocks of four k steps, two register buffers
    load(0, 0);
    for (int kb = 0; kb < nk; kb += 2) {
        if (kb + 1 < nk) load(1, (kb + 1) * 16);
        mma(0);
        if (kb + 1 >= nk) break;
        if (kb + 2 < nk) load(0, (kb + 2) * 16);
        mma(1);
    }
}

// U_b = D_b - sum_f O[b][f] (Rinv_r O[r][f^1]), r the red neighbour across
// face f.  One workgroup per black element; per face T = Rinv_r O[r][f^1] is
// formed in LDS, then O[b][f] T is subtracted from U, both on FP64 MFMA
// (tiles of 16 x 16, in groups of one row tile and up to three column
// tiles, dealt out to the wavefronts).  Each lane owns the same U entries
// for every face, and the first face starts from D_b.
__global__ void __launch_bounds__(kThreads) k_mb_schur(MeshK m, int nb, int nface, const double *__restrict__ D,
                                                       const double *__restrict__ O,
                                                       const double *__restrict__ Rinv, double *__restrict__ U) {
    extern __shared__ double T[];  // nb x nb, column-major
    const int c = blockIdx.x;
    const int k = colour_elem(m, c, 1);
    const int nn = nb * nb;
    const int nt = (nb + 15) / 16, njg = (nt + 2) / 3, ngroup = nt * njg;
    const int wave = threadIdx.x >> 6, nwave = blockDim.x >> 6;
    const int lane = threadIdx.x & 63, r16 = lane & 15, g = lane >> 4;
    double *u = U + (size_t)c * nn;
    const BlockRd Db(D + (size_t)k * nn, nb);
    for (int f = 0; f < nface; ++f) {
        const int r = neighbour(m, k, f >> 1, (f & 1) ? 1 : -1);
        const BlockRd Ri(Rinv + (size_t)(r >> 1) * nn, nb);
        const BlockRd Orb(O + ((size_t)r * nface + (f ^ 1)) * nn, nb);
        const BlockRd Obr(O + ((size_t)k * nface + f) * nn, nb);
        __syncthreads();  // the previous face's products have read T
        for (int gi = wave; gi < ngroup; gi += nwave) {
            const int it = gi / njg, jt0 = (gi % njg) * 3, nq = min(3, nt - jt0);
            f64x4_t acc[3];
#pragma unroll
            for (int q = 0; q < 3; ++q) acc[q] = f64x4_t{0.0, 0.0, 0.0, 0.0};
            schur_tiles(nb, it, jt0, nq, [&](int i, int kk) { return Ri.at(i, kk); },
                        [&](int kk, int j) { return Orb.at(kk, j); }, acc);
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                if (q >= nq) continue;
                const int j = (jt0 + q) * 16 + r16;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int i = it * 16 + g + 4 * v;
                    if (i < nb && j < nb) T[j * nb + i] = acc[q][v];
                }
            }
        }
        __syncthreads();
        for (int gi = wave; gi < ngroup; gi += nwave) {
            const int it = gi / njg, jt0 = (gi % njg) * 3, nq = min(3, nt - jt0);
            f64x4_t acc[3];
#pragma unroll
            for (int q = 0; q < 3; ++q) acc[q] = f64x4_t{0.0, 0.0, 0.0, 0.0};
            // B = T, read at clamped indices: its rows k >= nb meet zero A columns
            schur_tiles(nb, it, jt0, nq, [&](int i, int kk) { return Obr.at(i, kk); },
                        [&](int kk, int j) { return T[min(j, nb - 1) * nb + min(kk, nb - 1)]; }, acc);
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                if (q >= nq) continue;
                const int j = (jt0 + q) * 16 + r16;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int i = it * 16 + g + 4 * v;
                    if (i < nb && j < nb) {
                        const double prev = (f == 0) ? Db.at(i, j) : u[j * nb + i];
                        u[j * nb + i] = prev - acc[q][v];
                    }
                }
            }
        }
    }
}

enum RowMode { MB_MATVEC = 0, MB_INV = 1, MB_NBR_INV = 2, MB_MATVEC_BLACK = 3 };

// Block rows of the assembled operator, epb elements per workgroup:
//   MB_MATVEC : y_k = D_k x_k + sum_f O[k][f] x_nbr(k,f)          (every element)
//   MB_INV    : y_k = Inv_c r_k                                    (colour col)
//   MB_NBR_INV: y_k = Inv_c (r_k - sum_f O[k][f] x_nbr(k,f))       (colour col)
//   MB_MATVEC_BLACK: the product for x = (L U)^{-1} r: y_k = r_k on red
//               elements, where the factorisation keeps A's rows exactly
//               (L = I and U = A there), the product on black ones (pairs c)
// Inv holds one block per pair index c of the colour.  Each lane owns two
// consecutive rows of one element and reads them with one 16-byte load per
// block column (an odd block size, whose columns alternate 16-byte alignment,
// takes two 8-byte loads and leaves the last lane's second row empty); the columns of every block are split into S contiguous
// ranges on S lane groups (more lanes in flight on the small coarse level),
// whose partial sums meet in LDS and are added in range order.
template <int MODE, bool EVEN>
__global__ void __launch_bounds__(kThreads) k_mb_rows(MeshK m, int nb, int nface, int epb, int S, int col,
                                                      int count, const double *__restrict__ D,
                                                      const double *__restrict__ O,
                                                      const double *__restrict__ Inv, const double *x,
                                                      const double *__restrict__ r, double *y) {
    extern __shared__ double sh[];
    __shared__ int s_k[64];
    __shared__ int s_n[64][6];
    constexpr bool MV = (MODE == MB_MATVEC || MODE == MB_MATVEC_BLACK);
    const int nx = MV ? nface + 1 : nface;  // staged vectors per element
    double *s_x = sh;                                      // [epb][nx][nb]
    double *s_t = sh + (size_t)epb * (nface + 1) * nb;     // [epb][nb]
    double *s_p = s_t + (size_t)epb * nb;                  // [epb][S][nb] partial sums
    const int g0 = xcd_block(blockIdx.x, gridDim.x) * epb;
    const int ne = min(epb, count - g0);
    if ((int)threadIdx.x < ne) {
        const int g = g0 + threadIdx.x;
        const int k = (MODE == MB_MATVEC) ? g : colour_elem(m, g, col);
        s_k[threadIdx.x] = k;
        if (MODE != MB_INV)
            for (int f = 0; f < nface; ++f) s_n[threadIdx.x][f] = neighbour(m, k, f >> 1, (f & 1) ? 1 : -1);
    }
    __syncthreads();
    if (MODE != MB_INV) {
        for (int t = threadIdx.x; t < epb * nx * nb; t += blockDim.x) {
            const int e = t / (nx * nb);
            const int rem = t - e * nx * nb;
            const int f = rem / nb, j = rem - f * nb;
            double v = 0.0;
            if (e < ne) v = x[(size_t)j * m.Ne + (f < nface ? s_n[e][f] : s_k[e])];
            s_x[t] = v;
        }
    }
    if (MODE == MB_MATVEC_BLACK) {
        // the red element of each pair (k ^ 1): its rows of A z equal r
        for (int t = threadIdx.x; t < ne * nb; t += blockDim.x) {
            const int e = t / nb, j = t - e * nb;
            const size_t idx = (size_t)j * m.Ne + (s_k[e] ^ 1);
            y[idx] = r[idx];
        }
    }
    if (!MV) {
        for (int t = threadIdx.x; t < epb * nb; t += blockDim.x) {
            const int e = t / nb, j = t - e * nb;
            s_t[t] = (e < ne) ? r[(size_t)j * m.Ne + s_k[e]] : 0.0;
        }
    }
    __syncthreads();
    const int tpe = (nb + 1) / 2, lpe = tpe * S;
    const int e = threadIdx.x / lpe;
    const int rem = threadIdx.x - e * lpe;
    const int sg = rem / tpe;
    const int row = (rem - sg * tpe) * 2;
    const bool two = EVEN || row + 1 < nb;  // the lane's second row exists
    const bool active = e < ne;
    const int cs = (nb + S - 1) / S;
    const int j0 = min(nb, sg * cs), j1 = min(nb, j0 + cs);
    const size_t nn = (size_t)nb * nb;
    // partial sums of the S ranges, added in range order by group 0
    auto reduce = [&](double &a0, double &a1) {
        if (S == 1) return;
        if (active) {
            s_p[((size_t)e * S + sg) * nb + row] = a0;
            if (two) s_p[((size_t)e * S + sg) * nb + row + 1] = a1;
        }
        __syncthreads();
        if (active && sg == 0) {
            a0 = s_p[(size_t)e * S * nb + row];
            a1 = two ? s_p[(size_t)e * S * nb + row + 1] : 0.0;
            for (int q = 1; q < S; ++q) {
                a0 += s_p[((size_t)e * S + q) * nb + row];
                if (two) a1 += s_p[((size_t)e * S + q) * nb + row + 1];
            }
        }
        __syncthreads();
    };
    // two rows of column j: one 16-byte load, or two 8-byte ones (odd n_b)
    auto ld2 = [&](const double *p) -> double2 {
        if constexpr (EVEN) {
            return *reinterpret_cast<const double2 *>(p);
        } else {
            return double2{p[0], two ? p[1] : 0.0};
        }
    };
    auto gemv = [&](const double *blk, const double *xv, double &a0, double &a1) {
        blk += row;
        int j = j0;
        for (; j + 4 <= j1; j += 4) {
            const double2 v0 = ld2(blk + (size_t)j * nb);
            const double2 v1 = ld2(blk + (size_t)(j + 1) * nb);
            const double2 v2 = ld2(blk + (size_t)(j + 2) * nb);
            const double2 v3 = ld2(blk + (size_t)(j + 3) * nb);
            a0 += (v0.x * xv[j] + v1.x * xv[j + 1]) + (v2.x * xv[j + 2] + v3.x * xv[j + 3]);
            a1 += (v0.y * xv[j] + v1.y * xv[j + 1]) + (v2.y * xv[j + 2] + v3.y * xv[j + 3]);
        }
        for (; j < j1; ++j) {
            const double2 v0 = ld2(blk + (size_t)j * nb);
            a0 += v0.x * xv[j];
            a1 += v0.y * xv[j];
        }
    };
    double a0 = 0.0, a1 = 0.0;
    if (MODE != MB_INV) {
        if (active) {
            const int k = s_k[e];
            for (int f = 0; f < nx; ++f) {
                const double *blk = (f < nface) ? O + ((size_t)k * nface + f) * nn : D + (size_t)k * nn;
                gemv(blk, s_x + ((size_t)e * nx + f) * nb, a0, a1);
            }
        }
        reduce(a0, a1);
    }
    if (MV) {
        if (active && sg == 0) {
            const int k = s_k[e];
            y[(size_t)row * m.Ne + k] = a0;
            if (two) y[(size_t)(row + 1) * m.Ne + k] = a1;
        }
        return;
    }
    if (MODE == MB_NBR_INV && active && sg == 0) {
        s_t[e * nb + row] -= a0;
        if (two) s_t[e * nb + row + 1] -= a1;
    }
    __syncthreads();
    double b0 = 0.0, b1 = 0.0;
    if (active) gemv(Inv + (size_t)(g0 + e) * nn, s_t + e * nb, b0, b1);
    reduce(b0, b1);
    if (active && sg == 0) {
        const int k = s_k[e];
        y[(size_t)row * m.Ne + k] = b0;
        if (two) y[(size_t)(row + 1) * m.Ne + k] = b1;
    }
}

// ---------------------------------------------------------------------------
// GMRES cycle bookkeeping (one lane): Givens rotations of the Hessenberg
// column, convergence and breakdown, back substitution
// ---------------------------------------------------------------------------

__global__ void k_mb_gm_init(double *gm, double tol) {
    if (threadIdx.x != 0) return;
    const double beta = sqrt(gm[GM_N2]);
    for (int i = 0; i <= kMaxIt; ++i) gm[GM_G + i] = 0.0;
    gm[GM_G] = beta;
    gm[GM_TARGET] = tol * beta;
    gm[GM_DONE] = (beta == 0.0) ? 1.0 : 0.0;
    gm[GM_JEND] = 0.0;
}

__global__ void k_mb_gm_step(double *gm, int j, int m) {
    if (threadIdx.x != 0 || gm[GM_DONE] != 0.0) return;
    double *H = gm + GM_H;  // H[i + 9 jj]
    for (int i = 0; i <= j; ++i) H[i + 9 * j] = gm[GM_H1 + i] + gm[GM_H2 + i];
    const double hn = sqrt(gm[GM_N2]);
    H[j + 1 + 9 * j] = hn;
    for (int i = 0; i < j; ++i) {
        const double cs = gm[GM_CS + i], sn = gm[GM_SN + i];
        const double t = cs * H[i + 9 * j] + sn * H[i + 1 + 9 * j];
        H[i + 1 + 9 * j] = -sn * H[i + 9 * j] + cs * H[i + 1 + 9 * j];
        H[i + 9 * j] = t;
    }
    const double den = hypot(H[j + 9 * j], H[j + 1 + 9 * j]);
    const double cs = H[j + 9 * j] / den, sn = H[j + 1 + 9 * j] / den;
    gm[GM_CS + j] = cs;
    gm[GM_SN + j] = sn;
    H[j + 9 * j] = den;
    H[j + 1 + 9 * j] = 0.0;
    const double gj = gm[GM_G + j];
    gm[GM_G + j + 1] = -sn * gj;
    gm[GM_G + j] = cs * gj;
    const double res = fabs(gm[GM_G + j + 1]);
    if (hn == 0.0 || res <= gm[GM_TARGET] || j == m - 1) {
        gm[GM_DONE] = 1.0;
        gm[GM_JEND] = (double)(j + 1);
    }
}

__global__ void k_mb_gm_solve(double *gm) {
    if (threadIdx.x != 0) return;
    const int jend = (int)gm[GM_JEND];
    const double *H = gm + GM_H;
    for (int i = kMaxIt - 1; i >= 0; --i) {
        if (i >= jend) {
            gm[GM_Y + i] = 0.0;
            continue;
        }
        double t = gm[GM_G + i];
        for (int k = i + 1; k < jend; ++k) t -= H[i + 9 * k] * gm[GM_Y + k];
        gm[GM_Y + i] = t / H[i + 9 * i];
    }
}

// yout = yin - sum_{i < jend} y_i Z_i  (yin null: yout = the sum)
__global__ void __launch_bounds__(kThreads) k_mb_update(size_t n, const double *__restrict__ Z,
                                                        const double *__restrict__ gm, const double *yin,
                                                        double *yout) {
    const int jend = (int)gm[GM_JEND];
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x) {
        double d = 0.0;
        for (int i = 0; i < jend; ++i) d += gm[GM_Y + i] * Z[(size_t)i * n + t];
        yout[t] = yin ? yin[t] - d : d;
    }
}

unsigned grid_1d(size_t n) {
    const size_t g = (n + kThreads - 1) / kThreads;
    return (unsigned)std::min<size_t>(g, 8192);
}

// Column ranges per block: up to 4, while the launch has fewer than 256k
// lanes (4 wavefronts per SIMD) and every range keeps at least 4 columns.
int row_split(int nb, int count) {
    const int tpe = (nb + 1) / 2;
    int S = 1;
    while (S < 4 && (size_t)count * tpe * S < (256u << 10) && nb / (2 * S) >= 4 && tpe * 2 * S <= kThreads) S *= 2;
    return S;
}

template <int MODE>
hipError_t launch_rows(const frpmg_ctx *ctx, const Mbnk &mb, int col, const double *Inv, const double *x,
                       const double *r, double *y, hipStream_t s) {
    const int nb = mb.nb;
    if (nb < 4 || nb > kMbnkMaxNb) return hipErrorInvalidValue;
    const int count = (MODE == MB_MATVEC) ? mb.Ne : mb.Ne / 2;
    const int S = row_split(nb, MODE == MB_MATVEC_BLACK ? mb.Ne : count);
    const int lpe = ((nb + 1) / 2) * S;
    const int epb = std::min(64, std::max(1, kThreads / lpe));
    const size_t lds = ((size_t)epb * (mb.nface + 1) * nb + (size_t)epb * nb * (1 + S)) * sizeof(double);
    const dim3 grid((count + epb - 1) / epb);
    const dim3 block((epb * lpe + 63) / 64 * 64);
    if (nb % 2 == 0)
        hipLaunchKernelGGL((k_mb_rows<MODE, true>), grid, block, lds, s, ctx->mesh, nb, mb.nface, epb, S, col, count,
                           mb.D, mb.O, Inv, x, r, y);
    else
        hipLaunchKernelGGL((k_mb_rows<MODE, false>), grid, block, lds, s, ctx->mesh, nb, mb.nface, epb, S, col,
                           count, mb.D, mb.O, Inv, x, r, y);
    return hipGetLastError();
}

}  // namespace

hipError_t mb_perturb(const frpmg_ctx *ctx, const Mbnk &mb, const double *dq, int p0, int cnt, hipStream_t s) {
    const Level &L = ctx->lv[mb.level];
    if (cnt < 1 || (size_t)mb.nb * cnt > 65535) return hipErrorInvalidValue;
    const dim3 grid((ctx->mesh.Ne + kThreads - 1) / kThreads, mb.nb * cnt);
    hipLaunchKernelGGL(k_mb_perturb, grid, dim3(kThreads), 0, s, ctx->mesh, mb.nb, L.Np, ctx->phys, mb.stride[0],
                       mb.stride[1], mb.stride[2], p0, cnt, dq, mb.qb);
    return hipGetLastError();
}

hipError_t mb_extract(const frpmg_ctx *ctx, const Mbnk &mb, const double *dq, const double *r0, int p0, int cnt,
                        hipStream_t s) {
    const Level &L = ctx->lv[mb.level];
    const MeshK &m = ctx->mesh;
    int members = mb.nb;
    for (int a = 0; a < ctx->dim; ++a) members *= m.n[a] / mb.stride[a];
    if (cnt < 1 || (size_t)cnt * mb.nface > 65535) return hipErrorInvalidValue;
    const dim3 grid((members + kThreads - 1) / kThreads, cnt * mb.nface);
    hipLaunchKernelGGL(k_mb_extract, grid, dim3(kThreads), 0, s, m, mb.nb, L.Np, ctx->phys, mb.stride[0],
                       mb.stride[1], mb.stride[2], p0, cnt, mb.nface, dq, r0, mb.rb, mb.O);
    return hipGetLastError();
}

hipError_t mb_gather_red(const frpmg_ctx *ctx, const Mbnk &mb, hipStream_t s) {
    hipLaunchKernelGGL(k_mb_gather, dim3(mb.Ne / 2), dim3(kThreads), 0, s, ctx->mesh, mb.nb, 0, mb.D, mb.Rinv);
    return hipGetLastError();
}

hipError_t mb_schur(const frpmg_ctx *ctx, const Mbnk &mb, hipStream_t s) {
    const size_t lds = (size_t)mb.nb * mb.nb * sizeof(double);
    hipError_t e =
        hipFuncSetAttribute((const void *)k_mb_schur, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_mb_schur, dim3(mb.Ne / 2), dim3(kThreads), lds, s, ctx->mesh, mb.nb, mb.nface, mb.D, mb.O,
                       mb.Rinv, mb.Binv);
    return hipGetLastError();
}

hipError_t mb_matvec(const frpmg_ctx *ctx, const Mbnk &mb, const double *x, double *y, hipStream_t s) {
    return launch_rows<MB_MATVEC>(ctx, mb, 0, nullptr, x, nullptr, y, s);
}

hipError_t mb_ilu(const frpmg_ctx *ctx, const Mbnk &mb, const double *r, double *z, hipStream_t s) {
    hipError_t e = launch_rows<MB_INV>(ctx, mb, 0, mb.Rinv, nullptr, r, z, s);  // w_r = D_r^{-1} r_r
    if (e != hipSuccess) return e;
    e = launch_rows<MB_NBR_INV>(ctx, mb, 1, mb.Binv, z, r, z, s);  // z_b = U_b^{-1} (r_b - O_br w_r)
    if (e != hipSuccess) return e;
    return launch_rows<MB_NBR_INV>(ctx, mb, 0, mb.Rinv, z, r, z, s);  // z_r = D_r^{-1} (r_r - O_rb z_b)
}

hipError_t mb_sweep(frpmg_ctx *ctx, const Mbnk &mb, const double *G, const double *Yin, double *Yout, double tol,
                      int maxit, hipStream_t s) {
    if (maxit < 1 || maxit > kMaxIt || maxit > mb.mmax) return hipErrorInvalidValue;
    const size_t N = mb.N;
    double *gm = mb.gm;
    hipError_t e = vec_dot_normalize(ctx, N, G, gm + GM_N2, mb.V, s);  // v_0 = G / ||G||
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_mb_gm_init, dim3(1), dim3(64), 0, s, gm, tol);
    for (int j = 0; j < maxit; ++j) {
        double *vj = mb.V + (size_t)j * N;
        double *zj = mb.Z + (size_t)j * N;
        if ((e = mb_ilu(ctx, mb, vj, zj, s)) != hipSuccess) return e;
        // w = A z_j with z_j = (L U)^{-1} v_j: the red rows of A z_j are v_j's
        if ((e = launch_rows<MB_MATVEC_BLACK>(ctx, mb, 1, nullptr, zj, vj, mb.w, s)) != hipSuccess) return e;
        if ((e = vec_mdot(ctx, N, j + 1, mb.V, N, mb.w, gm + GM_H1, s)) != hipSuccess) return e;
        if ((e = vec_gemv_sub_mdot(ctx, N, j + 1, mb.V, N, gm + GM_H1, mb.w, gm + GM_H2, s)) != hipSuccess) return e;
        if ((e = vec_gemv_sub(N, j + 1, mb.V, N, gm + GM_H2, mb.w, s)) != hipSuccess) return e;
        if ((e = vec_dot_normalize(ctx, N, mb.w, gm + GM_N2, mb.V + (size_t)(j + 1) * N, s)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_mb_gm_step, dim3(1), dim3(64), 0, s, gm, j, maxit);
    }
    hipLaunchKernelGGL(k_mb_gm_solve, dim3(1), dim3(64), 0, s, gm);
    hipLaunchKernelGGL(k_mb_update, dim3(grid_1d(N)), dim3(kThreads), 0, s, N, mb.Z, gm, Yin, Yout);
    return hipGetLastError();
}

}  // namespace frpmg
