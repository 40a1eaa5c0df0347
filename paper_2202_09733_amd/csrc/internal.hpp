// Internal declarations of the frpmg library (gfx950).  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/frpmg.h"

namespace frpmg {

struct Lcc;
constexpr int kMaxP = 5;  // points per direction (p <= 4)

// 1D operators on [-1, 1] for one number of Gauss-Legendre points.
struct Ops1D {
    double D[kMaxP][kMaxP];  // D[i][j] = l_j'(xi_i)
    double bm[kMaxP];        // l_j(-1)
    double bp[kMaxP];        // l_j(+1)
    double gLd[kMaxP];       // derivative of the left correction at xi_i
    double gRd[kMaxP];       // derivative of the right correction at xi_i
    double dnp[kMaxP];       // sum_i l_i(+1) D[i][j]: derivative values interpolated to +1
    double cgp;              // sum_i l_i(+1) gRd[i]: right-correction derivative interpolated to +1
};

// 1D transfer operators between two levels (fine P0, coarse P1 points).
struct Transfer1D {
    int P0, P1;
    double G[kMaxP][kMaxP];   // restriction, P1 x P0
    double Pi[kMaxP][kMaxP];  // prolongation, P0 x P1
};

// Operators of every degree for meshes of mixed degree (p-adaptation):
// the 1D operators by point count, the 1D L2 projections between point
// counts (proj[Pa][Pb][b][a], from Pa to Pb points) and the Legendre
// coefficients of a P-point interpolant (modal[P][n][i]).
struct PaTables {
    Ops1D ops[kMaxP + 1];
    double proj[kMaxP + 1][kMaxP + 1][kMaxP][kMaxP];
    double modal[kMaxP + 1][kMaxP][kMaxP];
};

struct Phys {
    double gam, mu, Pr, tau;
    double qinf[5];
    double uinf[3];
    double pinf;
};

struct MeshK {
    int dim;
    int n[3];
    int Ne;
    const double *inv2h[3];  // device: 2 / h per axis index
    unsigned long long rcp[3];  // ceil(2^40 / n[a]): k / n[a] = (k rcp[a]) >> 40 while k n[a] < 2^40
};

// k / n[a] by the rounded-up reciprocal (exact while k n[a] < 2^40, which
// context creation checks): a multiply instead of a runtime division
__device__ __forceinline__ int div_axis(const MeshK &m, int k, int a) {
    return (int)(((unsigned long long)(unsigned)k * m.rcp[a]) >> 40);
}

// element coordinates; in 2D, c[2] numbers independent copies of the mesh
__device__ __forceinline__ void coords(const MeshK &m, int k, int c[3]) {
    const int r = div_axis(m, k, 0);
    c[0] = k - r * m.n[0];
    c[2] = div_axis(m, r, 1);
    c[1] = r - c[2] * m.n[1];
}

__device__ __forceinline__ int elem_index(const MeshK &m, const int c[3]) {
    return c[0] + m.n[0] * (c[1] + m.n[1] * c[2]);
}

// the element across the face normal to axis a on side s = -1 / +1 (periodic)
__device__ __forceinline__ int neighbour(const MeshK &m, int k, int a, int s) {
    int c[3];
    coords(m, k, c);
    int x = c[a] + s;
    if (x < 0) x += m.n[a];
    if (x >= m.n[a]) x -= m.n[a];
    c[a] = x;
    return elem_index(m, c);
}

// Finite-difference step of one perturbed entry: 1e-7 max(1, |q_inf + dq|).
__device__ __forceinline__ double fd_step(double qinf_v, double dqv) {
    return 1e-7 * fmax(1.0, fabs(qinf_v + dqv));
}

// Scalar that lives either on the host (p == nullptr) or in device memory.
// a scalar argument: the host value v, or m times the device value *p
struct Scal {
    double v;
    const double *p;
    double m = 1.0;
};

__device__ __forceinline__ double sval(const Scal &s) { return s.p ? s.m * *s.p : s.v; }

// How a residual launch forms the state it evaluates R at.
enum SrcMode { SRC_PLAIN = 0, SRC_AXPY = 1 };
// What a residual launch writes.
enum OutMode { OUT_R = 0, OUT_LIN = 1 };

struct ResidualArgs {
    SrcMode src = SRC_PLAIN;
    const double *dq = nullptr;   // base state deviation
    const double *v = nullptr;    // direction (SRC_AXPY)
    Scal alpha{1.0, nullptr};     // state = dq + alpha v
    OutMode out = OUT_R;
    double *r = nullptr;          // OUT_R / OUT_LIN destination
    const double *r0 = nullptr;   // OUT_LIN: R at the base state
    const double *x = nullptr;    // OUT_LIN: optional subtrahend
    double sigma = 0.0;           // OUT_LIN shift
    double dscale = 1.0;          // OUT_LIN: the difference is divided by dscale alpha
};

template <typename T>
struct DevBuf {
    T *p = nullptr;
    size_t n = 0;
};

// Mixed polynomial degrees on one level (p-adaptation, Sec. 3.3).  The
// level's P, Np, NF and nb are those of its largest degree; states, face
// arrays and EJ blocks keep that padded size.
struct PaLevel {
    std::vector<int> Pk_host;     // points per direction of every element
    int *Pk = nullptr;            // the same on the device [Ne]
    int *cls = nullptr;           // device: element ids grouped by point count
    int cls_off[kMaxP + 2] = {};  // class P is cls[cls_off[P] .. cls_off[P + 1])
    int *mixed = nullptr;         // device: faces between different degrees, k * 4 + a (k the -axis element)
    int nmixed = 0;
    double *Fm = nullptr;         // common flux on - faces at the element's points [dim][nv][NF][Ne]
    double *Mq = nullptr;         // mixed faces: the -axis element's + trace [dim][nv][NF][Ne]
    double *Mn = nullptr;         // mixed faces: the +axis element's - trace at its points [dim][nv][NF][Ne]
    double *Mg = nullptr;         // mixed faces: the -axis element's gradient trace [dim][dim][nv][NF][Ne]
    // EJ formation: fdB perturbed copies of the level evaluated together
    // (element id b Ne + k is element k of copy b); the lists and buffers
    // above, repeated per copy
    int fdB = 0;
    int *PkB = nullptr, *clsB = nullptr, *mixedB = nullptr;
    int clsB_off[kMaxP + 2] = {};
    double *JpB = nullptr, *FsB = nullptr, *FmB = nullptr, *MqB = nullptr, *MnB = nullptr, *MgB = nullptr;
    double *qB = nullptr, *rB = nullptr;  // [nv][Np][fdB Ne]
};

struct Level {
    PaLevel *pa = nullptr;  // mixed degrees (nullptr: every element has degree p)
    int p = 0, P = 0, Np = 0, NF = 0, nb = 0;
    size_t N = 0;  // state length
    Ops1D ops{};
    double *Jp = nullptr;  // state jumps q* - q+ on + faces [dim][nv][NF][Ne]
    double *Fs = nullptr;  // common fluxes on + faces [dim][nv][NF][Ne]
    // face data of the EJ linearisation point (allocated at the first factorisation)
    double *fQs = nullptr;  // q* on + faces [dim][nv][NF][Ne]
    double *fQp = nullptr;  // + traces [dim][nv][NF][Ne]
    double *fSn = nullptr;  // D part of the normal gradient at + faces [dim][nv][NF][Ne]
    double *fGt = nullptr;  // tangential gradients at + faces [dim][dim-1][nv][NF][Ne]
    // element-Jacobi storage: FP64 work blocks and the inverse
    double *blk64 = nullptr;  // [Ne][nb][nb], column-major per block
    void *inv = nullptr;      // inverse: points to blk64 (FP64) or inv32
    float *inv32 = nullptr;
    __bf16 *inv16 = nullptr;
    int inv_prec = -1;
    int *dstatus = nullptr;   // device pivot flags (kPivZero | kPivNonfinite)
    int *perm = nullptr;      // pivot rows of the blocked inversion [Ne][nb]
    int *touch = nullptr;     // touched-row lists of the blocked inversion [2][Ne][kTouchStride]
    int *colperm = nullptr;   // column placement of the blocked inversion [Ne][nb]
    const int *inv_cols = nullptr;  // nullptr: inv holds B^-1; else B^-1[:, inv_cols[j]] = inv[:, j]
    double *r0 = nullptr;     // scratch: R at the EJ linearisation point
};

// Workgroups are dispatched round-robin over the 8 XCDs of the chip, each
// with its own L2.  Remap the hardware workgroup index so that every XCD
// processes one contiguous range of logical workgroups: neighbouring
// elements then share their 128-byte lines and face data through one L2
// instead of each XCD fetching the same lines again.  A bijection on
// [0, nb).
__device__ __forceinline__ int xcd_block(int b, int nb) {
    constexpr int NX = 8;
    const int x = b % NX, j = b / NX;
    const int q = nb / NX, r = nb % NX;
    return (x < r) ? x * (q + 1) + j : r * (q + 1) + (x - r) * q + j;
}

// Blocked Gauss-Jordan: ints per block of one update window's touched-row
// list (the count, then up to 128 rows and the rows their values come from);
// each block holds two such lists.
constexpr int kTouchStride = 257;

// Reduction scratch: partial sums per block and per vector.
constexpr int kRedBlocks = 2048;     // capacity of the partial-sum buffer per vector
constexpr size_t kRedLarge = 4u << 20;  // vectors at least this long use up to kRedBlocks partials, others 512

// One captured Arnoldi step: the instantiated graph, the bit patterns of every
// parameter and pointer it bakes in, and the operation counts of one replay.
struct StepGraph {
    std::vector<unsigned long long> key;
    hipGraphExec_t exec = nullptr;
    long dR0 = 0, dR1 = 0, dE0 = 0, dE1 = 0;
};

// Matrix-based Newton-Krylov smoother of one level (Sec. 3.2): the
// assembled sigma I - dR/dq on the face-neighbour block pattern, its block
// ILU0 in red-black element order (colour = parity of the coordinate sum;
// with an even element count per axis, elements 2c and 2c + 1 take opposite
// colours, so c = k / 2 numbers each colour compactly), and the GMRES
// workspace.  Blocks are column-major, entry (row, col) at col nb + row.
struct Mbnk {
    int level = -1;
    int nb = 0, Ne = 0, nface = 0;
    size_t N = 0;
    double *D = nullptr;     // [Ne][nb][nb]: sigma I - dR_k/dq_k
    double *O = nullptr;     // [Ne][2 dim][nb][nb]: -dR_k/dq_m, m the face neighbour of slot 2a + (side > 0)
    double *Rinv = nullptr;  // [Ne/2][nb][nb]: D_k^{-1} of the red element of pair c
    double *Binv = nullptr;  // [Ne/2][nb][nb]: (D_b - sum_r O_br D_r^{-1} O_rb)^{-1} of the black element
    int stride[3] = {1, 1, 1};  // colouring of the neighbour-block differences
    int ncolour = 0;
    int batch = 0;           // perturbed copies per batched residual
    double *qb = nullptr, *rb = nullptr, *Jpb = nullptr, *Fsb = nullptr;
    int mmax = 0;            // GMRES workspace: basis V [mmax + 1][N], Z [mmax][N], w [N]
    double *V = nullptr, *Z = nullptr, *w = nullptr;
    double *gm = nullptr;    // device scalars of the GMRES cycle
    int *status = nullptr;
    bool allocated = false;  // every buffer above is in place
    bool ready = false;      // a factorisation is complete
};

}  // namespace frpmg

struct frpmg_ctx {
    int dim = 0, nv = 0, nlevels = 0;
    frpmg::MeshK mesh{};
    frpmg::Phys phys{};
    frpmg::Level lv[FR_MAX_LEVELS];
    frpmg::Transfer1D tr[FR_MAX_LEVELS];  // tr[l]: between level l and l + 1
    frpmg::PaTables *pa_tab = nullptr;       // device: operators of every degree (mixed-degree levels)
    frpmg::PaTables *pa_tab_host = nullptr;  // host copy
    double *inv2h[3] = {nullptr, nullptr, nullptr};
    std::string err;
    double *red_partial = nullptr;  // [128][kRedBlocks]
    double *red_out = nullptr;      // [64]
    double *scal = nullptr;         // device scalars [16]
    double *host_pinned = nullptr;   // pinned host staging [RO_SIZE]
    double *host_pinned2 = nullptr;  // second staging for an Arnoldi step launched ahead [RO_SIZE]
    double *noalloc_scratch = nullptr;  // this device's address of fr_residual_noalloc's array
    // preconditioner workspaces (allocated at creation)
    double *pq = nullptr, *prq = nullptr;    // linearisation point (borrowed pointers)
    double *q1 = nullptr, *r1 = nullptr;     // restricted point and R_1 there
    double *wY = nullptr, *wG = nullptr, *wXs = nullptr;
    double *cZ0 = nullptr, *cZ = nullptr, *cS = nullptr, *cG = nullptr, *cd = nullptr;
    // V-cycle work vectors of every coarse level l >= 1 (level 1: the names above)
    double *mq[FR_MAX_LEVELS] = {}, *mr[FR_MAX_LEVELS] = {}, *mZ0[FR_MAX_LEVELS] = {}, *mZ[FR_MAX_LEVELS] = {};
    double *mS[FR_MAX_LEVELS] = {}, *mG[FR_MAX_LEVELS] = {}, *md[FR_MAX_LEVELS] = {};
    const double *pt_q = nullptr, *pt_rq = nullptr;
    // Krylov workspaces (allocated at the first stage solve)
    int kdim = 0;
    double *V = nullptr, *Zk = nullptr, *kw = nullptr;
    double *sq = nullptr, *srq = nullptr, *sF = nullptr, *sb = nullptr, *sdx = nullptr;
    double *stv = nullptr, *stw = nullptr;  // time step: stage vectors [stv_n][N], state scratch
    int stv_n = 0;
    // learned coarse correction (allocated on first use)
    frpmg::Lcc *lcc = nullptr;
    // MBNK smoother (allocated at the first mbnk_factor)
    frpmg::Mbnk *mb = nullptr;
    // per-phase timing of host-launched Arnoldi steps (events created at the first stage solve):
    // preconditioner, FD product, orthogonalisation and normalisation, seconds summed over a stage
    // (one set of four per buffer of two Arnoldi steps in flight)
    hipEvent_t ph_ev[8] = {};
    hipEvent_t step_ev[2] = {};  // an Arnoldi step's Hessenberg column has reached its pinned staging
    double ph_acc[3] = {0.0, 0.0, 0.0};
    // captured Arnoldi steps, replayed on the caller's stream
    hipStream_t cap_stream = nullptr;
    std::vector<frpmg::StepGraph> graphs;
    unsigned long long graph_epoch = 0;  // bumped whenever baked-in factors change
};

namespace frpmg {

// ops1d.cpp
void build_ops1d(int P, Ops1D &o);
void build_transfer(int P0, int P1, Transfer1D &t);
void build_pa_tables(PaTables &t);
void gauss_legendre(int P, double *x, double *w);

// residual.hip
hipError_t launch_residual(const frpmg_ctx *ctx, int level, const ResidualArgs &a, hipStream_t s);
// r0 = R(dq) and the FP64 blocks sigma I - dR_k/dq_k of every element into
// out (null: L.blk64), [Ne][nb][nb] column-major per block
hipError_t launch_ej_form(const frpmg_ctx *ctx, int level, const double *dq, double sigma, hipStream_t s,
                          double *out = nullptr);
// r = R(dq) for `batch` independent copies of a 2D level's state, copy b at
// elements b Ne .. (b + 1) Ne - 1 of [nv][Np][batch Ne] arrays; face buffers
// Jp and Fs hold [dim][nv][NF][batch Ne].  3D: batch must be 1.
// mixed-degree levels (residual.hip)
hipError_t launch_residual_pa(const frpmg_ctx *ctx, int level, const ResidualArgs &a, hipStream_t s);
hipError_t launch_ej_form_pa(const frpmg_ctx *ctx, int level, const double *dq, double sigma, hipStream_t s,
                             double *out);
hipError_t pa_transfer(const frpmg_ctx *ctx, int from, int to, const double *x, double *y, const double *x0,
                       bool accumulate, const double *x2, double *y2, hipStream_t s);
hipError_t pa_project(const frpmg_ctx *ctx, const int *deg_from, int NpF, const double *x, const int *deg_to,
                      int NpT, double *y, hipStream_t s);
hipError_t pa_indicator(const frpmg_ctx *ctx, int level, const double *dq, int var, double *eta, hipStream_t s);
hipError_t pa_adapt(const frpmg_ctx *ctx, const double *eta, const int *deg_in, int *deg_out, int p_min, int p_max,
                    double nu_max, double nu_min, hipStream_t s);
hipError_t launch_residual_batch(const frpmg_ctx *ctx, int level, int batch, const double *dq, double *r,
                                 double *Jp, double *Fs, hipStream_t s);

// vec.hip
hipError_t vec_dot(frpmg_ctx *ctx, size_t n, const double *x, const double *y, double *dout, hipStream_t s);
hipError_t vec_mdot(frpmg_ctx *ctx, size_t n, int nvec, const double *V, size_t ldv, const double *w,
                    double *dout, hipStream_t s);
hipError_t vec_gemv_sub(size_t n, int nvec, const double *V, size_t ldv, const double *h, double *w,
                        hipStream_t s);
// w -= V h, then dout = V^T w (the updated w), in one pass over V; the same
// bits as vec_gemv_sub followed by vec_mdot
hipError_t vec_gemv_sub_mdot(frpmg_ctx *ctx, size_t n, int nvec, const double *V, size_t ldv, const double *h,
                             double *w, double *dout, hipStream_t s);
// y = a x + b y (a, b host or device scalars); x may be null (then y = b y)
hipError_t vec_axpby(size_t n, Scal a, const double *x, Scal b, double *y, hipStream_t s);
// y = a x
hipError_t vec_scale_copy(size_t n, Scal a, const double *x, double *y, hipStream_t s);
// y = x0 + sum_i c[i] Z_i  with host coefficients
hipError_t vec_combine(size_t n, int nvec, const double *Z, size_t ldz, const double *c_dev, double *y,
                       hipStream_t s);
hipError_t vec_fill(size_t n, double v, double *y, hipStream_t s);
// y = x / sqrt(n2) with the squared norm n2 on the device
hipError_t vec_normalize(size_t n, const double *n2, const double *x, double *y, hipStream_t s);
// out = (x - b) * c - r   (stage function)
hipError_t vec_stage_F(size_t n, const double *x, const double *b, double c, const double *r, double *out,
                       hipStream_t s);
// FD step h = eps (1 + ||dq||) / ||v|| from squared norms on the device
// (dqn2 = null drops the state size)
hipError_t scal_fd_step(const double *vn2, const double *dqn2, double eps, double *hout, hipStream_t s);
// preconditioner scale s = eps_p sigma (1 + ||q||) / ||X|| and 1/s (qn2 = null drops the state size)
hipError_t scal_pmg_scale(const double *xn2, const double *qn2, double eps_p, double sigma, double *s_out,
                          double *inv_out, hipStream_t s);
// y = T x (or y += T (x - x0) with x0 / accumulate), T = restriction or prolongation
// restriction of two vectors in one launch: y = Gamma x, y2 = Gamma x2
hipError_t transfer_restrict2(const frpmg_ctx *ctx, int fine_level, const double *x, double *y, const double *x2,
                              double *y2, hipStream_t s);
hipError_t transfer_apply(const frpmg_ctx *ctx, int fine_level, bool restrict_dir, const double *x,
                          double *y, hipStream_t s, const double *x0 = nullptr, bool accumulate = false);
// ||v||^2 -> n2out and the FD step h = eps (1 + ||dq||) / ||v|| -> hout, one reduction
hipError_t vec_dot_fd_step(frpmg_ctx *ctx, size_t n, const double *v, const double *dqn2, double eps,
                           double *n2out, double *hout, hipStream_t s);
// ||x||^2 -> n2out and y = x / ||x||, one reduction
hipError_t vec_dot_normalize(frpmg_ctx *ctx, size_t n, const double *x, double *n2out, double *y, hipStream_t s);
// ||X||^2 -> n2out and the preconditioner scale s, 1/s, one reduction
hipError_t vec_dot_pmg_scale(frpmg_ctx *ctx, size_t n, const double *x, const double *qn2, double eps_p,
                             double sigma, double *n2out, double *s_out, double *inv_out, hipStream_t s);

// ej.hip
// pivot flags the inversion kernels OR into their status word
constexpr int kPivZero = 1;       // an exact zero pivot
constexpr int kPivNonfinite = 2;  // a NaN or infinite pivot
// true when the blocks of this size and precision take the blocked inversion
bool ej_blocked(int nb, int precision);
hipError_t ej_invert(frpmg_ctx *ctx, int level, int precision, hipStream_t s);
// out[i] = in[i]^{-1} for `count` FP64 blocks of nb <= 128 (LDS Gauss-Jordan,
// partial pivoting, exact column order); the pivot flags are ORed into
// *status.  in may equal out.
hipError_t invert_blocks_f64(int count, int nb, const double *in, double *out, int *status, hipStream_t s);

// mbnk.hip
constexpr int kMbnkMaxIt = 8;
// largest MBNK block (the 3D p = 2 coarse level has 135 unknowns per element);
// its LDS Gauss-Jordan and Schur products keep a whole FP64 block in LDS
constexpr int kMbnkMaxNb = 136;
// colour-batch kernels of the neighbour-block formation: pairs p0 .. p0 + cnt - 1
// (pair = colour nb + column) perturbed into qb ([nv][Np][cnt Ne]); their
// residuals rb extracted into the off-diagonal blocks
hipError_t mb_perturb(const frpmg_ctx *ctx, const Mbnk &mb, const double *dq, int p0, int cnt, hipStream_t s);
hipError_t mb_extract(const frpmg_ctx *ctx, const Mbnk &mb, const double *dq, const double *r0, int p0, int cnt,
                        hipStream_t s);
// Rinv = red D blocks (inverted by the caller); Binv = black Schur complements
hipError_t mb_gather_red(const frpmg_ctx *ctx, const Mbnk &mb, hipStream_t s);
hipError_t mb_schur(const frpmg_ctx *ctx, const Mbnk &mb, hipStream_t s);
// y = A x on the assembled pattern
hipError_t mb_matvec(const frpmg_ctx *ctx, const Mbnk &mb, const double *x, double *y, hipStream_t s);
// z = (L U)^{-1} r, three element-parallel steps; z must not alias r
hipError_t mb_ilu(const frpmg_ctx *ctx, const Mbnk &mb, const double *r, double *z, hipStream_t s);
// Yout = Yin - delta (Yin null: Yout = delta), delta ~ A^{-1} G by
// right-ILU0-preconditioned GMRES(maxit <= kMbnkMaxIt) to relative tolerance
// tol, every decision taken on the device.  G may alias Yin or Yout.
hipError_t mb_sweep(frpmg_ctx *ctx, const Mbnk &mb, const double *G, const double *Yin, double *Yout, double tol,
                      int maxit, hipStream_t s);
// y = beta y + alpha B^{-1} r
hipError_t ej_apply(const frpmg_ctx *ctx, int level, const double *r, double alpha, double beta, double *y,
                    hipStream_t s);
// y = scale (beta yin + alpha B^{-1} r); yin may be y
hipError_t ej_apply_ex(const frpmg_ctx *ctx, int level, const double *r, double alpha, double beta,
                       const double *yin, Scal scale, double *y, hipStream_t s);

}  // namespace frpmg
