// Element-Jacobi blocks on gfx950: inversion of every block (Sec. 2.2,
// element-Jacobi preconditioner; Sec. 3.2, EJ smoother).  The batched apply
// with the stored inverses is in ej_apply.hip.
//
// Inversion of small blocks (EJ blocks of n_b <= 64: 2D up to p = 3, 3D
// p <= 1; the kernel takes up to 128): one workgroup per block, the whole
// FP64 block resident in LDS, Gauss-Jordan elimination with partial pivoting
// (largest |a|, first row on ties), the inverse written back column-major in
// the requested storage precision.  Larger blocks (2D p = 4 and 3D from
// p = 2: an LDS-resident 135^2 block leaves one workgroup per CU and ran 4x
// slower than the blocked form, 100^2 blocks 2x), and the BF16-MFMA precision
// form at any size, use the blocked variant below.  Storing the inverse turns every
// apply into a batched GEMV that streams the blocks once from HBM with
// coalesced column reads, with no sequential triangular sweeps.
#include <cfloat>
#include <utility>

#include "internal.hpp"

namespace frpmg {

namespace {

constexpr int kGJThreads = 256;
constexpr int kMaxLdsBlock = kMbnkMaxNb;  // LDS form: EJ blocks up to 64, MBNK blocks up to 136 (147 KB of LDS)

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
    int flags = 0;
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
            // a column of NaNs compares false everywhere: keep row c
            if (ii < c || ii >= nb) ii = c;
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
            flags |= kPivZero;
            d = 1.0;
        } else if (!(fabs(d) <= DBL_MAX)) {
            flags |= kPivNonfinite;
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
    if (flags && tid == 0) atomicOr(status, flags);
}

// ---------------------------------------------------------------------------
// Blocked in-place Gauss-Jordan for the larger blocks (100 x 100 in 2D at
// p = 4; 135 x 135 and 320 x 320 in 3D at p = 2, 3).  Sub-panels of kPanel
// columns are eliminated in registers (pivot search over the full column,
// row swaps recorded).  The product of a window's elementary transforms is
// T = (I + W S^T) P (S = the window's pivot rows), and applying it to any
// other column is one GEMM:
//     x <- (P x with the pivot rows zeroed) + T_win (P x)_S,
// where T_win = the window's columns as the elimination left them.  Two
// sub-panels form one window of kWide columns: the first sub-panel's
// transform is applied to the second sub-panel's columns only, the second
// is eliminated, its transform is applied to the first sub-panel's columns
// only, and the combined transform then updates every other column in one
// pass -- half the passes over the block set that one update per sub-panel
// takes, with the same elimination steps.  The row interchanges turn into
// column interchanges of the result, which are not carried out: the column
// placement is recorded and the apply gathers r through it.
// ---------------------------------------------------------------------------
constexpr int kPanel = 32;                    // columns of one register sub-panel
constexpr int kWide = 2 * kPanel;             // columns of one update window
constexpr int kMaxNb = 512;                   // largest block the blocked form takes
constexpr int kTouch = 2 * kWide;             // S plus at most one moved row per pivot step
static_assert(kTouchStride == 1 + 2 * kTouch, "touched-row list: count, rows[kTouch], sources[kTouch]");

// The panel kernel also tracks which input row each lane's values came from;
// at the end it writes the list of touched rows (the window rows S in order,
// then every other row whose content moved, with its source row) that the
// update kernels use to apply the interchanges to the other columns as a
// gather.  A row outside S that moved holds the former content of a row of
// S (contents leave S only by a swap with a later pivot row), so its source
// lies inside the window's rows.

// Panel factorisation with the panel in registers, NW wavefronts per block
// (NW = 2..4): lane t of the workgroup owns rows t, t + 64 NW, ... (kPanel
// values each, RPL rows), so a pivot step needs two barriers whatever NW is.
// Per step: each wavefront's argmax by shuffles (the lowest row wins ties),
// combined through LDS (barrier); the owners of the pivot row and of row c
// put them in LDS (barrier); every lane swaps and eliminates its rows against
// the pivot row, read column by column from LDS.  The steps are instantiated
// per panel column so that every register index is a constant (a runtime
// index would put the rows in scratch memory).  At most two rows per lane
// (64 doubles) keep the rows in registers without spilling; a block of 320
// rows takes three wavefronts of two rows per lane (3.2 ms per launch on
// 32,768 blocks, against 3.5 ms for two wavefronts of three rows, which
// spill, and 5.0 ms for five wavefronts of one row, whose steps wait longer
// at the barriers).  Outputs: the panel columns in place, the pivot rows,
// the touched-row lists and the pivot flags.
constexpr int kPanel2MaxWaves = 4;

struct Panel2Lds {
    double v[kPanel2MaxWaves];
    int i[kPanel2MaxWaves];
    int cnt[2][kPanel2MaxWaves];
    int porg, corg, porg2, corg2;
    double pivrow[kPanel];
    double oldc[kPanel];
    short upos[kMaxNb];  // the first sub-panel's list: slot of row r (-1: untouched)
    int tsrc[kTouch];
};

template <int RPL, int NW, int CC>
__device__ __forceinline__ void panel2_step(double (&x)[RPL][kPanel], int (&org)[RPL], int (&org2)[RPL],
                                            Panel2Lds &sh, int t, int nb, int c0, int bw, int *__restrict__ perm,
                                            int &flags) {
    constexpr int NT = 64 * NW;
    if (CC >= bw) return;
    const int c = c0 + CC;
    double best = -1.0;
    int bi = 0x7fffffff;
#pragma unroll
    for (int s = 0; s < RPL; ++s) {
        const int r = s * NT + t;
        if (r >= c && r < nb) argmax_combine(best, bi, fabs(x[s][CC]), r);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const double v2 = __shfl_xor(best, off, 64);
        const int i2 = __shfl_xor(bi, off, 64);
        argmax_combine(best, bi, v2, i2);
    }
    if ((t & 63) == 0) {
        sh.v[t >> 6] = best;
        sh.i[t >> 6] = bi;
    }
    __syncthreads();
    double bv = sh.v[0];
    int p = sh.i[0];
#pragma unroll
    for (int w = 1; w < NW; ++w) argmax_combine(bv, p, sh.v[w], sh.i[w]);
    if (p < c || p >= nb) p = c;  // a column of NaNs compares false everywhere: keep row c
    if (t == 0) perm[(size_t)blockIdx.x * nb + c] = p;
    const int sp = p / NT, tp = p - sp * NT;
    const int sc = c / NT, tc = c - sc * NT;
#pragma unroll
    for (int s = 0; s < RPL; ++s) {
        if (s == sp && t == tp) {
#pragma unroll
            for (int j = 0; j < kPanel; ++j) sh.pivrow[j] = x[s][j];
            sh.porg = org[s];
            sh.porg2 = org2[s];
        }
        if (s == sc && t == tc && p != c) {
#pragma unroll
            for (int j = 0; j < kPanel; ++j) sh.oldc[j] = x[s][j];
            sh.corg = org[s];
            sh.corg2 = org2[s];
        }
    }
    __syncthreads();
    if (p != c) {
#pragma unroll
        for (int s = 0; s < RPL; ++s) {
            if (s == sp && t == tp) {
#pragma unroll
                for (int j = 0; j < kPanel; ++j) x[s][j] = sh.oldc[j];
                org[s] = sh.corg;
                org2[s] = sh.corg2;
            }
            if (s == sc && t == tc) {
                org[s] = sh.porg;
                org2[s] = sh.porg2;
            }
        }
    }
    double d = sh.pivrow[CC];
    if (d == 0.0) {
        flags |= kPivZero;
        d = 1.0;
    } else if (!(fabs(d) <= DBL_MAX)) {
        flags |= kPivNonfinite;
    }
    const double inv = 1.0 / d;
    // every row: x - f pv with f its multiplier (column CC: -f / d); rows
    // beyond the block compute values nobody stores; row c then takes the
    // scaled pivot row (one lane)
    double f[RPL];
#pragma unroll
    for (int s = 0; s < RPL; ++s) f[s] = x[s][CC];
#pragma unroll
    for (int j = 0; j < kPanel; ++j) {
        const double pv = (j == CC ? 1.0 : sh.pivrow[j]) * inv;
#pragma unroll
        for (int s = 0; s < RPL; ++s) x[s][j] = (j == CC ? 0.0 : x[s][j]) - f[s] * pv;
    }
    // the pivot row is read again below: keep the compiler from holding it in
    // registers across the loop (it would not fit beside the rows)
    __asm__ volatile("" ::: "memory");
    if (t == tc) {
#pragma unroll
        for (int s = 0; s < RPL; ++s) {
            if (s == sc) {
#pragma unroll
                for (int j = 0; j < kPanel; ++j) x[s][j] = (j == CC ? 1.0 : sh.pivrow[j]) * inv;
            }
        }
    }
}

template <int RPL, int NW, int... CC>
__device__ __forceinline__ void panel2_steps(std::integer_sequence<int, CC...>, double (&x)[RPL][kPanel],
                                             int (&org)[RPL], int (&org2)[RPL], Panel2Lds &sh, int t, int nb,
                                             int c0, int bw, int *__restrict__ perm, int &flags) {
    (panel2_step<RPL, NW, CC>(x, org, org2, sh, t, nb, c0, bw, perm, flags), ...);
}

// Write the touched-row list of the window [lo, lo + w) from the lanes' row
// origins: slot r - lo for the window rows, then the moved rows in row
// order, ranked by wavefront ballots per slot (rows s*64NW + t: slot major,
// then wavefront, then lane).  Every lane takes part; starts with a barrier.
template <int RPL, int NW>
__device__ __forceinline__ void write_touch(const int (&org)[RPL], int lo, int w, int nb, int t, Panel2Lds &sh,
                                            int *__restrict__ tl) {
    constexpr int NT = 64 * NW;
    const int lane = t & 63, wv = t >> 6;
    unsigned long long m[RPL];
    __syncthreads();  // the previous readers of sh.cnt are done
#pragma unroll
    for (int s = 0; s < RPL; ++s) {
        const int r = s * NT + t;
        const bool inS = r >= lo && r < lo + w;
        m[s] = __ballot(r < nb && !inS && org[s] != r);
        if (lane == 0) sh.cnt[s][wv] = __popcll(m[s]);
    }
    __syncthreads();
    int off = w;
#pragma unroll
    for (int s = 0; s < RPL; ++s) {
        const int r = s * NT + t;
        const bool inS = r >= lo && r < lo + w;
        int base = off, all = 0;
#pragma unroll
        for (int u = 0; u < NW; ++u) {
            base += u < wv ? sh.cnt[s][u] : 0;
            all += sh.cnt[s][u];
        }
        int slot = -1;
        if (inS)
            slot = r - lo;
        else if ((m[s] >> lane) & 1ull)
            slot = base + __popcll(m[s] & ((1ull << lane) - 1ull));
        if (slot >= 0) {
            tl[1 + slot] = r;
            tl[1 + kTouch + slot] = org[s];
        }
        off += all;
    }
    if (t == 0) tl[0] = off;
}

// One sub-panel [c0, c0 + bw) of every block.  wlo == c0: a window of its
// own; its list goes to touch.  wlo < c0: the second sub-panel of the
// window [wlo, c0 + bw), whose first sub-panel's list is read from touch
// (before it is overwritten with this sub-panel's own list); the list of the
// whole window, with the interchanges of both sub-panels composed, goes to
// touch2.
template <int RPL, int NW>
__global__ void __launch_bounds__(64 * NW)
k_gj_panel2(int nb, int c0, int bw, int wlo, double *__restrict__ A, int *__restrict__ perm,
            int *__restrict__ touch, int *__restrict__ touch2, int *__restrict__ status) {
    static_assert(RPL <= 2 && NW >= 2 && NW <= kPanel2MaxWaves, "rows per lane, wavefronts per block");
    constexpr int NT = 64 * NW;
    __shared__ Panel2Lds sh;
    const int t = threadIdx.x;
    const bool second = wlo < c0;
    double *Ak = A + (size_t)blockIdx.x * nb * nb;
    int *tl = touch + (size_t)blockIdx.x * kTouchStride;
    if (second) {
        for (int r = t; r < nb; r += NT) sh.upos[r] = -1;
        __syncthreads();
        const int nu = min(tl[0], kTouch);
        for (int u = t; u < nu; u += NT) {
            const int r = tl[1 + u];
            if (r >= 0 && r < nb) sh.upos[r] = (short)u;
            sh.tsrc[u] = tl[1 + kTouch + u];
        }
        __syncthreads();
    }
    double x[RPL][kPanel];
    int org[RPL], org2[RPL];
#pragma unroll
    for (int s = 0; s < RPL; ++s) {
        const int r = s * NT + t;
        org[s] = r;
        const int u = (second && r < nb) ? sh.upos[r] : -1;
        org2[s] = u >= 0 ? sh.tsrc[u] : r;
#pragma unroll
        for (int j = 0; j < kPanel; ++j) x[s][j] = (r < nb && j < bw) ? Ak[(size_t)(c0 + j) * nb + r] : 0.0;
    }
    int flags = 0;
    panel2_steps<RPL, NW>(std::make_integer_sequence<int, kPanel>{}, x, org, org2, sh, t, nb, c0, bw, perm, flags);
#pragma unroll
    for (int s = 0; s < RPL; ++s) {
        const int r = s * NT + t;
        if (r < nb) {
#pragma unroll
            for (int j = 0; j < kPanel; ++j)
                if (j < bw) Ak[(size_t)(c0 + j) * nb + r] = x[s][j];
        }
    }
    write_touch<RPL, NW>(org, c0, bw, nb, t, sh, tl);
    if (second) write_touch<RPL, NW>(org2, wlo, c0 + bw - wlo, nb, t, sh, touch2 + (size_t)blockIdx.x * kTouchStride);
    if (flags && t == 0) atomicOr(status, flags);
}

constexpr int kUpdCols = 64;  // columns per update workgroup
constexpr int kUpdRows = 64;  // rows per chunk

// The window's touched-row list of one block in LDS: (P x)[rows[u]] =
// x[src[u]], upos[r] = slot of row r (-1: untouched, (P x)[r] = x[r]).
struct TouchLds {
    int rows[kTouch];
    int src[kTouch];
    short upos[kMaxNb];
    int nu;
};

// The columns an update launch transforms: tile column ri < n is block column
// j = lo + ri, shifted past the excluded window [skip_lo, skip_lo + skip_w)
// (the window's own columns).
struct ColMap {
    int lo, n, skip_lo, skip_w;
    __device__ __forceinline__ int col(int ri) const {
        const int j = lo + ri;
        return j >= skip_lo ? j + skip_w : j;
    }
};

// Workgroup -> (block, column tile).  Workgroups are dispatched round-robin
// over the 8 XCDs; block k goes to XCD k mod 8 and its column tiles run back
// to back there, so the window columns they all read stay in that XCD's L2.
__device__ __forceinline__ bool update_tile(int Ne, int ntile, int &k, int &tile) {
    const int g = blockIdx.x, xcd = g & 7, i = g >> 3;
    k = (i / ntile) * 8 + xcd;
    tile = i - (i / ntile) * ntile;
    return k < Ne;
}

// Load block k's touched-row list; every lane takes part, ends with a barrier.
__device__ __forceinline__ void load_touch(TouchLds &t, const int *__restrict__ tl, int nb) {
    const int tid = threadIdx.x;
    for (int r = tid; r < nb; r += blockDim.x) t.upos[r] = -1;
    const int nu = min(tl[0], kTouch);
    if (tid < nu) {
        t.rows[tid] = tl[1 + tid];
        t.src[tid] = tl[1 + kTouch + tid];
    }
    if (tid == 0) t.nu = nu;
    __syncthreads();
    if (tid < nu) t.upos[t.rows[tid]] = (short)tid;
    __syncthreads();
}

// stg[jj][u] = (P x_j)_S[u] = x_j[src[u]] for the window rows u < bw and the
// tile's columns (0 beyond), the operand of the product.  Read before any
// write of the tile.
template <int KP, typename Buf>
__device__ __forceinline__ void stage_window_rows(const TouchLds &t, double (*stg)[KP + 1], const Buf &B, int nb,
                                                  const ColMap &cm, int tile, int bw) {
    for (int i = threadIdx.x; i < KP * kUpdCols; i += blockDim.x) {
        const int u = i % KP, jj = i / KP;
        const int ri = tile * kUpdCols + jj;
        const bool ok = u < bw && ri < cm.n;
        stg[jj][u] = B.ld(Buf::at(cm.col(ri) * nb + t.src[ok ? u : 0], ok));
    }
}

// Row chunks in the order an update stores them: the chunk that holds the
// window rows S last (the window starts at a multiple of kPanel and spans at
// most kWide rows, so S lies in one chunk).  Every moved row outside S reads
// its source inside S, so up to the last chunk no store overwrites a value
// still to be read; the last chunk's own reads finish before a barrier that
// precedes its stores.
__device__ __forceinline__ int chunk_row(int i, int nch, int cs) {
    const int c = (i == nch - 1) ? cs : (i < cs ? i : i + 1);
    return c * kUpdRows;
}

typedef double f64x4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

// Lane geometry shared by the update kernels.  They form the product
// transposed, out^T = (P x)_S^T T_win^T, on 16 x 16 MFMA tiles: wave w owns
// rows wave*16 + r16 of each 64-row chunk, and lane (r16, g) holds the
// results of that row in 16 columns of the tile: cb*16 + 4g + v for the
// FP32-output MFMA, cb*16 + g + 4v for the FP64 one (cb, v < 4).  Each store
// instruction therefore writes four 128-byte column segments.
template <bool F64>
struct UpdLane {
    int r16, g, wave;
    int ri0, c0, bw;  // c0, bw: the window (its columns hold T, its rows are S)
    ColMap cm;
    __device__ UpdLane(int tid, int tile, const ColMap &cm_, int c0_, int bw_) {
        const int lane = tid & 63;
        wave = tid >> 6;
        r16 = lane & 15;
        g = lane >> 4;
        ri0 = tile * kUpdCols;
        cm = cm_;
        c0 = c0_;
        bw = bw_;
    }
    // tile column of result (cb, v)
    __device__ __forceinline__ int jj(int cb, int v) const { return cb * 16 + (F64 ? g + 4 * v : 4 * g + v); }
    // its block column; false beyond the launch's columns
    __device__ __forceinline__ bool col(int cb, int v, int &j) const {
        const int ri = ri0 + jj(cb, v);
        j = cm.col(ri);
        return ri < cm.n;
    }
};

// Block-relative buffer addressing for the update kernels: every read and
// write is issued unconditionally, and a lane with nothing to read or write
// passes an offset beyond the block, which the buffer range check turns into
// a zero read or a dropped write.  With no branches around memory
// instructions the compiler waits for exactly the reads a use needs.
typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));
constexpr unsigned kOutside = 0x80000000u;  // byte offset beyond every block (n_b <= 512: 2 MB)
constexpr int kBufWord3 = 0x00020000;       // buffer descriptor word 3: 32-bit data format, no swizzle
struct BlockBuf {
    __amdgpu_buffer_rsrc_t rs;
    __device__ BlockBuf(double *Ak, int nb)
        : rs(__builtin_amdgcn_make_buffer_rsrc(Ak, (short)0, nb * nb * (int)sizeof(double), kBufWord3)) {}
    __device__ __forceinline__ static unsigned at(int idx, bool ok) {
        return ok ? (unsigned)idx * (unsigned)sizeof(double) : kOutside;
    }
    __device__ __forceinline__ double ld(unsigned off) const {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0));
    }
    __device__ __forceinline__ void st(unsigned off, double v) const {
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, v), rs, off, 0, 0);
    }
};

// The global reads of one 64-row chunk, issued ahead of their use: the
// chunk of the window columns T (KP/4 values per lane, rows fastest; issued
// before the previous chunk's product) and the lane's (P x) values (issued
// right after the previous chunk's stores; none on the window rows, whose
// output is the product alone).  Reads outside the window's columns or the
// block's rows return 0.
template <int KP>
struct ChunkLoads {
    double tpv[KP / 4];
    double xo[4][4];
    template <bool F64>
    __device__ void issue_t(const BlockBuf &B, const UpdLane<F64> &L, int nb, int r0) {
        const int tid = threadIdx.x;
#pragma unroll
        for (int i = 0; i < KP / 4; ++i) {
            const int t = tid + 256 * i, cc = t >> 6, rr = t & 63;
            tpv[i] = B.ld(BlockBuf::at((L.c0 + cc) * nb + r0 + rr, cc < L.bw && r0 + rr < nb));
        }
    }
    // tp[cc][rr] = T[r0 + rr][cc]
    __device__ void put_t(double (*tp)[kUpdRows]) const {
        const int tid = threadIdx.x;
#pragma unroll
        for (int i = 0; i < KP / 4; ++i) {
            const int t = tid + 256 * i;
            tp[t >> 6][t & 63] = tpv[i];
        }
    }
    template <bool F64>
    __device__ void issue_x(const BlockBuf &B, const TouchLds &tl, const UpdLane<F64> &L, int nb, int r0) {
        const int r = r0 + L.wave * 16 + L.r16;
        const bool row = r < nb && !(r >= L.c0 && r < L.c0 + L.bw);
        const int u = r < nb ? tl.upos[r] : -1;
        const int rs = u >= 0 ? tl.src[u] : r;
#pragma unroll
        for (int cb = 0; cb < 4; ++cb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                int j;
                const bool ok = L.col(cb, v, j);
                xo[cb][v] = B.ld(BlockBuf::at(j * nb + rs, row && ok));
            }
    }
};

// Write the lane's results of one chunk: out = (P x, zero on S) + product.
template <bool F64, typename Acc>
__device__ __forceinline__ void store_chunk(const BlockBuf &B, const UpdLane<F64> &L, const double (&xo)[4][4],
                                            const Acc &acc, int nb, int r0) {
    const int r = r0 + L.wave * 16 + L.r16;
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            int j;
            const bool ok = L.col(cb, v, j);
            B.st(BlockBuf::at(j * nb + r, ok && r < nb), xo[cb][v] + acc[cb][v]);
        }
}

// Before the last chunk's stores: every lane's reads are complete (the last
// chunk's moved rows read window rows that the same chunk overwrites).
__device__ __forceinline__ void reads_done_barrier() {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
}

// Apply a window's transform (K = KP: one sub-panel, or two as one window)
// to kUpdCols columns (outside the window) of one block in FP64 on
// v_mfma_f64_16x16x4f64 (A = stage^T: lane (r16, g) gives column r16, window
// column 4ks + g; B = T^T: window column 4ks + g, row r16).  The next chunk's
// global reads are in flight while a chunk is multiplied.
template <int KP>
__device__ __forceinline__ void gj_update_f64(int Ne, int nb, int c0, int bw, const ColMap &cm,
                                              double *__restrict__ A, const int *__restrict__ touch,
                                              double (*stg)[KP + 1], double (*tp)[kUpdRows], TouchLds &tl) {
    const int ntile = (cm.n + kUpdCols - 1) / kUpdCols;
    int k, tile;
    if (!update_tile(Ne, ntile, k, tile)) return;
    const int tid = threadIdx.x;
    const BlockBuf B(A + (size_t)k * nb * nb, nb);
    load_touch(tl, touch + (size_t)k * kTouchStride, nb);
    stage_window_rows<KP>(tl, stg, B, nb, cm, tile, bw);
    const UpdLane<true> L(tid, tile, cm, c0, bw);
    const int nch = (nb + kUpdRows - 1) / kUpdRows, cs = c0 / kUpdRows;
    ChunkLoads<KP> ld;
    ld.issue_t(B, L, nb, chunk_row(0, nch, cs));
    ld.issue_x(B, tl, L, nb, chunk_row(0, nch, cs));
    for (int i = 0; i < nch; ++i) {
        const int r0 = chunk_row(i, nch, cs);
        __syncthreads();  // the stage is complete; the previous chunk's tp reads are done
        ld.put_t(tp);
        __syncthreads();
        const bool more = i + 1 < nch;
        const int r1 = more ? chunk_row(i + 1, nch, cs) : 0;
        if (more) ld.issue_t(B, L, nb, r1);
        f64x4_t acc[4];
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) acc[cb] = f64x4_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int ks = 0; ks < KP / 4; ++ks) {
            const double bv = tp[4 * ks + L.g][L.wave * 16 + L.r16];
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) {
                const double av = stg[cb * 16 + L.r16][4 * ks + L.g];
                acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[cb], 0, 0, 0);
            }
        }
        if (!more) reads_done_barrier();
        store_chunk(B, L, ld.xo, acc, nb, r0);
        if (more) ld.issue_x(B, tl, L, nb, r1);
    }
}

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
k_gj_update(int Ne, int nb, int c0, int bw, ColMap cm, double *__restrict__ A, const int *__restrict__ touch) {
    __shared__ double stg[kUpdCols][kPanel + 1];  // (P x)_S
    __shared__ double tp[kPanel][kUpdRows];       // T chunk, [window column][row]
    __shared__ TouchLds tl;
    gj_update_f64<kPanel>(Ne, nb, c0, bw, cm, A, touch, stg, tp, tl);
}

// The whole-window update (K = kWide); 69 KB of LDS, two workgroups per CU.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
k_gj_update_wide(int Ne, int nb, int c0, int bw, ColMap cm, double *__restrict__ A, const int *__restrict__ touch) {
    __shared__ double stg[kUpdCols][kWide + 1];
    __shared__ double tp[kWide][kUpdRows];
    __shared__ TouchLds tl;
    gj_update_f64<kWide>(Ne, nb, c0, bw, cm, A, touch, stg, tp, tl);
}

// The update on BF16-input MFMA with FP32 accumulation
// (v_mfma_f32_16x16x32_bf16, K = 32 per instruction: one sub-panel, or two
// steps for a whole window): each FP32 operand is split into hi + lo BF16
// parts and the product taken as hi*hi + lo*hi + hi*lo (three MFMAs), ~16
// mantissa bits.  Operands are staged k-contiguous in LDS (rows padded by 8
// values to spread the 16-byte reads over the banks).
template <int KP>
__device__ __forceinline__ void gj_update_bf16(int Ne, int nb, int c0, int bw, const ColMap &cm,
                                               double *__restrict__ A, const int *__restrict__ touch,
                                               __bf16 (*xs_h)[KP + 8], __bf16 (*xs_l)[KP + 8],
                                               __bf16 (*tp_h)[KP + 8], __bf16 (*tp_l)[KP + 8], TouchLds &tl) {
    const int ntile = (cm.n + kUpdCols - 1) / kUpdCols;
    int k, tile;
    if (!update_tile(Ne, ntile, k, tile)) return;
    const int tid = threadIdx.x;
    const BlockBuf B(A + (size_t)k * nb * nb, nb);
    load_touch(tl, touch + (size_t)k * kTouchStride, nb);
    // (P x)_S of the tile's columns, split into hi and lo parts
    for (int i = tid; i < KP * kUpdCols; i += 256) {
        const int u = i % KP, jj = i / KP;
        const int ri = tile * kUpdCols + jj;
        const bool ok = u < bw && ri < cm.n;
        const float v = (float)B.ld(BlockBuf::at(cm.col(ri) * nb + tl.src[ok ? u : 0], ok));
        const __bf16 h = (__bf16)v;
        xs_h[jj][u] = h;
        xs_l[jj][u] = (__bf16)(v - (float)h);
    }
    const UpdLane<false> L(tid, tile, cm, c0, bw);
    const int nch = (nb + kUpdRows - 1) / kUpdRows, cs = c0 / kUpdRows;
    ChunkLoads<KP> ld;
    ld.issue_t(B, L, nb, chunk_row(0, nch, cs));
    ld.issue_x(B, tl, L, nb, chunk_row(0, nch, cs));
    for (int i = 0; i < nch; ++i) {
        const int r0 = chunk_row(i, nch, cs);
        __syncthreads();  // xs is complete; the previous chunk's tp reads are done
#pragma unroll
        for (int q = 0; q < KP / 4; ++q) {
            const int t = tid + 256 * q, cc = t >> 6, rr = t & 63;
            const float v = (float)ld.tpv[q];
            const __bf16 h = (__bf16)v;
            tp_h[rr][cc] = h;
            tp_l[rr][cc] = (__bf16)(v - (float)h);
        }
        __syncthreads();
        const bool more = i + 1 < nch;
        const int r1 = more ? chunk_row(i + 1, nch, cs) : 0;
        if (more) ld.issue_t(B, L, nb, r1);
        f32x4_t acc[4];
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) acc[cb] = f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kk = 0; kk < KP / 32; ++kk) {
            const int k8 = 32 * kk + 8 * L.g;
            const bf16x8_t th = *reinterpret_cast<const bf16x8_t *>(&tp_h[L.wave * 16 + L.r16][k8]);
            const bf16x8_t tlo = *reinterpret_cast<const bf16x8_t *>(&tp_l[L.wave * 16 + L.r16][k8]);
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) {
                const bf16x8_t xh = *reinterpret_cast<const bf16x8_t *>(&xs_h[cb * 16 + L.r16][k8]);
                const bf16x8_t xl = *reinterpret_cast<const bf16x8_t *>(&xs_l[cb * 16 + L.r16][k8]);
                acc[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh, th, acc[cb], 0, 0, 0);
                acc[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xl, th, acc[cb], 0, 0, 0);
                acc[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh, tlo, acc[cb], 0, 0, 0);
            }
        }
        if (!more) reads_done_barrier();
        store_chunk(B, L, ld.xo, acc, nb, r0);
        if (more) ld.issue_x(B, tl, L, nb, r1);
    }
}

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
k_gj_update_mfma(int Ne, int nb, int c0, int bw, ColMap cm, double *__restrict__ A, const int *__restrict__ touch) {
    __shared__ __attribute__((aligned(16))) __bf16 xs_h[kUpdCols][kPanel + 8];
    __shared__ __attribute__((aligned(16))) __bf16 xs_l[kUpdCols][kPanel + 8];
    __shared__ __attribute__((aligned(16))) __bf16 tp_h[kUpdRows][kPanel + 8];
    __shared__ __attribute__((aligned(16))) __bf16 tp_l[kUpdRows][kPanel + 8];
    __shared__ TouchLds tl;
    gj_update_bf16<kPanel>(Ne, nb, c0, bw, cm, A, touch, xs_h, xs_l, tp_h, tp_l, tl);
}

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
k_gj_update_mfma_wide(int Ne, int nb, int c0, int bw, ColMap cm, double *__restrict__ A,
                      const int *__restrict__ touch) {
    __shared__ __attribute__((aligned(16))) __bf16 xs_h[kUpdCols][kWide + 8];
    __shared__ __attribute__((aligned(16))) __bf16 xs_l[kUpdCols][kWide + 8];
    __shared__ __attribute__((aligned(16))) __bf16 tp_h[kUpdRows][kWide + 8];
    __shared__ __attribute__((aligned(16))) __bf16 tp_l[kUpdRows][kWide + 8];
    __shared__ TouchLds tl;
    gj_update_bf16<kWide>(Ne, nb, c0, bw, cm, A, touch, xs_h, xs_l, tp_h, tp_l, tl);
}

// The row interchanges of the elimination turn into column interchanges of
// the result (undone last first).  Instead of moving columns, record where
// each stored column belongs: the inverse is X[:, sigma(j)] = A[:, j], so
// X r = sum_j A[:, j] r[sigma(j)] and the apply reads r through sigma.  One
// lane composes the interchanges in LDS; the others fill and write out.
__global__ void __launch_bounds__(64) k_gj_colperm(int nb, const int *__restrict__ perm, int *__restrict__ sigma) {
    __shared__ int pi[kMaxNb];  // pi[c] = stored column that becomes column c of X
    __shared__ int pv[kMaxNb];
    const int tid = threadIdx.x;
    const size_t base = (size_t)blockIdx.x * nb;
    for (int c = tid; c < nb; c += blockDim.x) {
        pi[c] = c;
        pv[c] = perm[base + c];
    }
    __syncthreads();
    if (tid == 0) {
        for (int c = nb - 1; c >= 0; --c) {
            const int p = pv[c];
            if (p != c) {
                const int t = pi[c];
                pi[c] = pi[p];
                pi[p] = t;
            }
        }
    }
    __syncthreads();
    for (int c = tid; c < nb; c += blockDim.x) sigma[base + pi[c]] = c;
}

// Narrow storage of the blocked inversion's result: stored column j of
// block k is column sigma[k][j] of the inverse, so the conversion writes it
// there and the narrow apply needs no column gather (64x64 p = 4, BF16:
// 17.2 -> 16.1 us per fine apply).
template <typename T>
__global__ void k_to_narrow_placed(int Ne, int nb, const double *__restrict__ a, const int *__restrict__ sigma,
                                   T *__restrict__ b) {
    const size_t nn = (size_t)nb * nb, n = nn * Ne;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride) {
        const size_t k = t / nn, rem = t - k * nn;
        const int j = (int)(rem / nb), i = (int)(rem - (size_t)j * nb);
        b[k * nn + (size_t)sigma[k * nb + j] * nb + i] = (T)(float)a[t];
    }
}

}  // namespace

// Blocks above 64 unknowns take the blocked form in every precision: at 4096
// blocks of 100^2 it inverts in 1.8 ms where the LDS form, one workgroup per
// block, takes 3.5 ms; the apply's column gather costs 0.5 us of 56.
constexpr int kLdsMaxPreferred = 64;

bool ej_blocked(int nb, int precision) {
    return nb > kLdsMaxPreferred || precision == FR_PREC_FP32_BF16 || precision == FR_PREC_BF16_STORE;
}

hipError_t invert_blocks_f64(int count, int nb, const double *in, double *out, int *status, hipStream_t s) {
    if (nb > kMaxLdsBlock || count < 0) return hipErrorInvalidValue;
    if (count == 0) return hipSuccess;
    const size_t lds = ((size_t)nb * nb + nb) * sizeof(double);
    hipError_t e = hipFuncSetAttribute((const void *)k_gj_invert<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_gj_invert<double>, dim3(count), dim3(kGJThreads), lds, s, nb, in, out, status);
    return hipGetLastError();
}

hipError_t ej_invert(frpmg_ctx *ctx, int level, int precision, hipStream_t s) {
    Level &L = ctx->lv[level];
    const int nb = L.nb, Ne = ctx->mesh.Ne;
    if (ej_blocked(nb, precision)) {
        if (nb > kMaxNb || !L.perm || !L.touch || !L.colperm) return hipErrorInvalidValue;
        const bool mfma = precision == FR_PREC_FP32_BF16 || precision == FR_PREC_BF16_STORE;
        // rows per lane x wavefronts of the panel kernel: one row per lane up
        // to 256 rows, two above
        auto panel = [&](int c, int bw, int wlo, int *touch, int *touch2) {
            const dim3 gp(Ne);
#define FR_PANEL2(R, W)                                                                                        \
    hipLaunchKernelGGL((k_gj_panel2<R, W>), gp, dim3(64 * W), 0, s, nb, c, bw, wlo, L.blk64, L.perm, touch, touch2, \
                       L.dstatus)
            if (nb <= 128)
                FR_PANEL2(1, 2);
            else if (nb <= 192)
                FR_PANEL2(1, 3);
            else if (nb <= 256)
                FR_PANEL2(1, 4);
            else if (nb <= 384)
                FR_PANEL2(2, 3);
            else
                FR_PANEL2(2, 4);
#undef FR_PANEL2
        };
        auto grid = [&](const ColMap &cm) {
            const int ntile = (cm.n + kUpdCols - 1) / kUpdCols;
            return dim3((unsigned)(((Ne + 7) / 8) * 8 * ntile));
        };
        // one sub-panel's transform applied to the columns cm lists
        auto update = [&](int c, int bw, const ColMap &cm, const int *touch) {
            if (cm.n <= 0) return;
            if (mfma)
                hipLaunchKernelGGL(k_gj_update_mfma, grid(cm), dim3(256), 0, s, Ne, nb, c, bw, cm, L.blk64, touch);
            else
                hipLaunchKernelGGL(k_gj_update, grid(cm), dim3(256), 0, s, Ne, nb, c, bw, cm, L.blk64, touch);
        };
        int *tsub = L.touch, *twin = L.touch + (size_t)Ne * kTouchStride;
        constexpr int kNever = kMaxNb;  // ColMap without an excluded window
        for (int c0 = 0; c0 < nb; c0 += kWide) {
            const int bw1 = min(kPanel, nb - c0), bw2 = min(kPanel, nb - c0 - bw1);
            panel(c0, bw1, c0, tsub, nullptr);
            if (bw2 <= 0) {
                update(c0, bw1, ColMap{0, nb - bw1, c0, bw1}, tsub);
                continue;
            }
            update(c0, bw1, ColMap{c0 + bw1, bw2, kNever, 0}, tsub);  // first transform on the second sub-panel
            panel(c0 + bw1, bw2, c0, tsub, twin);
            update(c0 + bw1, bw2, ColMap{c0, bw1, kNever, 0}, tsub);  // second transform on the first sub-panel
            const int bw = bw1 + bw2;
            const ColMap cm{0, nb - bw, c0, bw};
            if (cm.n <= 0) continue;
            if (mfma)
                hipLaunchKernelGGL(k_gj_update_mfma_wide, grid(cm), dim3(256), 0, s, Ne, nb, c0, bw, cm, L.blk64,
                                   twin);
            else
                hipLaunchKernelGGL(k_gj_update_wide, grid(cm), dim3(256), 0, s, Ne, nb, c0, bw, cm, L.blk64, twin);
        }
        hipLaunchKernelGGL(k_gj_colperm, dim3(Ne), dim3(64), 0, s, nb, L.perm, L.colperm);
        if (precision == FR_PREC_FP64) {
            L.inv = L.blk64;
            L.inv_cols = L.colperm;  // the apply gathers r through the placement
        } else if (precision == FR_PREC_BF16_STORE) {
            hipLaunchKernelGGL(k_to_narrow_placed<__bf16>, dim3(4096), dim3(256), 0, s, Ne, nb, L.blk64, L.colperm,
                               L.inv16);
            L.inv = L.inv16;
            L.inv_cols = nullptr;
        } else {
            hipLaunchKernelGGL(k_to_narrow_placed<float>, dim3(4096), dim3(256), 0, s, Ne, nb, L.blk64, L.colperm,
                               L.inv32);
            L.inv = L.inv32;
            L.inv_cols = nullptr;
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
    L.inv_cols = nullptr;
    L.inv_prec = precision;
    return hipGetLastError();
}

}  // namespace frpmg
