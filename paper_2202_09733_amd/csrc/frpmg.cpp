// Host orchestration of the frpmg library: context set-up, the C ABI entry
// points, the nonlinear p-multigrid V-cycle (Sec. 3.1 applied as the
// preconditioner of Sec. 3.2), flexible GMRES with classical Gram-Schmidt
// and one re-orthogonalisation, and the ESDIRK / ROW stage drivers
// (Sec. 2.1, 2.2).  All vector work runs in the HIP kernels of residual.hip,
// vec.hip and ej.hip; the host only sequences launches and runs the small
// Hessenberg least-squares problem.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <functional>
#include <mutex>
#include <random>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "internal.hpp"
#include "lcc.hpp"

using namespace frpmg;

namespace {

struct Fail {
    fr_status code;
};

#define HIPCHK(expr)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess) {                                                               \
            ctx->err = std::string(#expr) + ": " + hipGetErrorString(e_);                     \
            throw Fail{e_ == hipErrorOutOfMemory ? FR_ENOMEM : FR_EDEVICE};                   \
        }                                                                                     \
    } while (0)

#define REQUIRE(cond, msg)              \
    do {                                \
        if (!(cond)) {                  \
            ctx->err = (msg);           \
            throw Fail{FR_EINVAL};      \
        }                               \
    } while (0)

template <typename F>
fr_status guarded(frpmg_ctx *ctx, F &&f) {
    if (!ctx) return FR_EINVAL;
    try {
        f();
        return FR_OK;
    } catch (const Fail &x) {
        return x.code;
    } catch (const std::bad_alloc &) {
        ctx->err = "host allocation failed";
        return FR_ENOMEM;
    }
}

// Scratch of fr_residual_noalloc, for callers that cannot allocate: the
// face data that the face kernel hands to the volume kernel (common fluxes
// and state jumps on each element's + faces).  Every device the library
// runs on holds its own copy until the process ends.  Host code never passes
// the symbol itself to a kernel: each device's address is taken once, with
// that device current, at fr_create.
constexpr size_t kNoallocBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) double scratch[kNoallocBytes / sizeof(double)];
std::mutex g_scratch_mu;
double *g_scratch_addr[kMaxDevices] = {};

double *dalloc(frpmg_ctx *ctx, size_t n) {
    void *p = nullptr;
    HIPCHK(hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(double)));
    return (double *)p;
}

void dfree(void *p) {
    if (p) (void)hipFree(p);
}

hipStream_t S(fr_stream s) { return (hipStream_t)s; }

// a named range on the profiler's timeline (roctx; no cost without a profiler)
struct Range {
    explicit Range(const char *name) { roctxRangePushA(name); }
    ~Range() { roctxRangePop(); }
    Range(const Range &) = delete;
    Range &operator=(const Range &) = delete;
};

int ipow(int b, int e) {
    int r = 1;
    while (e--) r *= b;
    return r;
}

// ---- device scalars (slots of ctx->scal) ----
enum { SC_JVP_H = 0, SC_JVP_N2 = 1, SC_PMG_S = 2, SC_PMG_INV = 3, SC_PMG_N2 = 4, SC_DQ_N2 = 5, SC_PT_N2 = 6 };
// ---- reduction outputs (slots of ctx->red_out) ----
constexpr int kMaxKdim = 120;  // Krylov dimension cap: m + 1 <= 128 dot products per pass
constexpr int RO_H1 = 0, RO_H2 = 128, RO_Y = 256, RO_N2 = 384, RO_SIZE = 512;

// operation counts of a stage solve (fine / coarse residuals, EJ applies)
struct Counters {
    long R0 = 0, R1 = 0, E0 = 0, E1 = 0;
};

double host_norm(frpmg_ctx *ctx, size_t n, const double *x, hipStream_t s) {
    HIPCHK(vec_dot(ctx, n, x, x, ctx->red_out + RO_N2, s));
    HIPCHK(hipMemcpyAsync(ctx->host_pinned, ctx->red_out + RO_N2, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return std::sqrt(ctx->host_pinned[0]);
}

void residual(frpmg_ctx *ctx, int level, const double *dq, double *r, hipStream_t s) {
    ResidualArgs a;
    a.src = SRC_PLAIN;
    a.dq = dq;
    a.out = OUT_R;
    a.r = r;
    HIPCHK(launch_residual(ctx, level, a, s));
}

// out = sigma v - (R(dq + alpha v) - r0) / (dscale alpha) - x   (x optional)
void residual_lin(frpmg_ctx *ctx, int level, const double *dq, const double *v, Scal alpha, const double *r0,
                  double sigma, const double *x, double *out, hipStream_t s, double dscale = 1.0) {
    ResidualArgs a;
    a.src = SRC_AXPY;
    a.dq = dq;
    a.v = v;
    a.alpha = alpha;
    a.out = OUT_LIN;
    a.r = out;
    a.r0 = r0;
    a.x = x;
    a.sigma = sigma;
    a.dscale = dscale;
    HIPCHK(launch_residual(ctx, level, a, s));
}

bool valid_eps_mode(int mode) {
    const int step = mode & ~FR_FD_CENTRAL;
    return step >= FR_EPS_ABSOLUTE && step <= FR_EPS_SCALED;
}

// One-sided: w = shift v - (R(dq + h v) - rq) / h.  With FR_FD_CENTRAL in
// mode: w = shift v - (R(dq + h v) - R(dq - h v)) / (2 h) (rq unused; the
// level's V-cycle G vector holds R(dq - h v)).  dqn2: device ||dq||^2 for
// the SCALED step (computed here when null).
void jvp(frpmg_ctx *ctx, int level, const double *dq, const double *rq, const double *v, double shift,
         double eps, int mode, double *w, hipStream_t s, const double *dqn2 = nullptr) {
    const bool central = (mode & FR_FD_CENTRAL) != 0;
    mode &= ~FR_FD_CENTRAL;
    Scal h{eps, nullptr};
    const size_t N = ctx->lv[level].N;
    if (mode == FR_EPS_NORMALIZED || mode == FR_EPS_SCALED) {
        const double *size = nullptr;
        if (mode == FR_EPS_SCALED) {
            if (!dqn2) {
                HIPCHK(vec_dot(ctx, N, dq, dq, ctx->scal + SC_DQ_N2, s));
                dqn2 = ctx->scal + SC_DQ_N2;
            }
            size = dqn2;
        }
        HIPCHK(vec_dot_fd_step(ctx, N, v, size, eps, ctx->scal + SC_JVP_N2, ctx->scal + SC_JVP_H, s));
        h = Scal{0.0, ctx->scal + SC_JVP_H};
    }
    if (!central) {
        residual_lin(ctx, level, dq, v, h, rq, shift, nullptr, w, s);
        return;
    }
    double *rm = level == 0 ? ctx->wG : ctx->mG[level];
    ResidualArgs a;
    a.src = SRC_AXPY;
    a.dq = dq;
    a.v = v;
    a.alpha = Scal{-h.v, h.p, -1.0};
    a.out = OUT_R;
    a.r = rm;
    HIPCHK(launch_residual(ctx, level, a, s));
    residual_lin(ctx, level, dq, v, h, rm, shift, nullptr, w, s, 2.0);
}

// The element-local block formation takes the face neighbours as
// unperturbed: each must differ from the element itself.
void check_neighbours(frpmg_ctx *ctx) {
    for (int a = 0; a < ctx->dim; ++a)
        REQUIRE(ctx->mesh.n[a] >= 2, "EJ formation needs at least two elements per axis");
}

// face data of a level's linearisation point, kept by the element-local block formation
void ensure_face_save(frpmg_ctx *ctx, Level &L) {
    const size_t nface = (size_t)ctx->dim * ctx->nv * L.NF * ctx->mesh.Ne;
    if (!L.fQs) L.fQs = dalloc(ctx, nface);
    if (!L.fQp) L.fQp = dalloc(ctx, nface);
    if (!L.fSn) L.fSn = dalloc(ctx, nface);
    if (!L.fGt) L.fGt = dalloc(ctx, nface * (ctx->dim - 1));
}

void ej_factor_impl(frpmg_ctx *ctx, int level, const double *dq, double sigma, int precision, hipStream_t s) {
    Range range(level == 0 ? "ej_factor level 0" : "ej_factor coarse level");
    REQUIRE(level >= 0 && level < ctx->nlevels, "bad level");
    REQUIRE(precision >= FR_PREC_FP64 && precision <= FR_PREC_BF16_STORE, "bad precision");
    check_neighbours(ctx);
    Level &L = ctx->lv[level];
    REQUIRE(L.nb <= 512, "EJ block too large (n_b > 512)");
    const size_t nblk = (size_t)ctx->mesh.Ne * L.nb * L.nb;
    if (!L.blk64) L.blk64 = dalloc(ctx, nblk);
    if (ej_blocked(L.nb, precision) && !L.perm) {
        void *p = nullptr;
        HIPCHK(hipMalloc(&p, (size_t)ctx->mesh.Ne * L.nb * sizeof(int)));
        L.perm = (int *)p;
        HIPCHK(hipMalloc(&p, (size_t)ctx->mesh.Ne * 2 * kTouchStride * sizeof(int)));
        L.touch = (int *)p;
        HIPCHK(hipMalloc(&p, (size_t)ctx->mesh.Ne * L.nb * sizeof(int)));
        L.colperm = (int *)p;
    }
    if ((precision == FR_PREC_FP32 || precision == FR_PREC_FP32_BF16) && !L.inv32) {
        void *p = nullptr;
        HIPCHK(hipMalloc(&p, nblk * sizeof(float)));
        L.inv32 = (float *)p;
    }
    if (precision == FR_PREC_BF16_STORE && !L.inv16) {
        void *p = nullptr;
        HIPCHK(hipMalloc(&p, nblk * sizeof(__bf16)));
        L.inv16 = (__bf16 *)p;
    }
    if (L.pa) {
        for (int a = 0; a < ctx->dim; ++a)
            REQUIRE(ctx->mesh.n[a] % 2 == 0, "EJ formation on a mixed-degree level needs even element counts");
    } else {
        ensure_face_save(ctx, L);
    }
    ctx->graph_epoch++;  // captured steps bake in the factor buffers and precision
    HIPCHK(hipMemsetAsync(L.dstatus, 0, sizeof(int), s));
    HIPCHK(launch_ej_form(ctx, level, dq, sigma, s));
    HIPCHK(ej_invert(ctx, level, precision, s));
    int flag = 0;
    HIPCHK(hipMemcpyAsync(ctx->host_pinned, L.dstatus, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    std::memcpy(&flag, ctx->host_pinned, sizeof(int));
    if (flag & kPivNonfinite) {
        ctx->err = "non-finite pivot in an element-Jacobi block (NaN or Inf in the blocks)";
        throw Fail{FR_ENONFINITE};
    }
    if (flag) {
        ctx->err = "zero pivot in an element-Jacobi block";
        throw Fail{FR_ESINGULAR};
    }
}


// ---------------------------------------------------------------------------
// MBNK smoother (Sec. 3.2): assembled face-neighbour Jacobian, red-black
// block ILU0, GMRES sweeps
// ---------------------------------------------------------------------------

constexpr size_t kMbnkBatchDoubles = size_t(1) << 24;  // perturbed states per batched residual (128 MiB)
constexpr int kMbnkGm = 256;                           // device scalars of the GMRES cycle

void mbnk_free(frpmg_ctx *ctx) {
    Mbnk *mb = ctx->mb;
    if (!mb) return;
    double *bufs[] = {mb->D, mb->O, mb->Rinv, mb->Binv, mb->qb, mb->rb, mb->Jpb, mb->Fsb, mb->V, mb->Z, mb->w, mb->gm};
    for (double *b : bufs) dfree(b);
    dfree(mb->status);
    delete mb;
    ctx->mb = nullptr;
}

// Smallest divisor of n that is at least 3: elements of one colour are then
// at least three apart along the axis, across the periodic wrap too.
int colour_stride(int n) {
    for (int s = 3; s <= n; ++s)
        if (n % s == 0) return s;
    return 0;
}

void mbnk_alloc(frpmg_ctx *ctx, int level) {
    if (ctx->mb && ctx->mb->level == level && ctx->mb->allocated) return;
    mbnk_free(ctx);  // also a workspace left partial by a failed allocation
    const Level &L = ctx->lv[level];
    const MeshK &m = ctx->mesh;
    Mbnk *mb = new Mbnk();
    ctx->mb = mb;
    mb->level = level;
    mb->nb = L.nb;
    mb->Ne = m.Ne;
    mb->nface = 2 * ctx->dim;
    mb->N = L.N;
    mb->ncolour = 1;
    for (int a = 0; a < ctx->dim; ++a) {
        mb->stride[a] = colour_stride(m.n[a]);
        mb->ncolour *= mb->stride[a];
    }
    const size_t nn = (size_t)L.nb * L.nb;
    mb->D = dalloc(ctx, (size_t)m.Ne * nn);
    mb->O = dalloc(ctx, (size_t)m.Ne * mb->nface * nn);
    mb->Rinv = dalloc(ctx, (size_t)(m.Ne / 2) * nn);
    mb->Binv = dalloc(ctx, (size_t)(m.Ne / 2) * nn);
    // 2D: as many perturbed copies per launch as fit the batch budget, the
    // launch grids and the element-index range; 3D: one copy
    int batch = 1;
    if (ctx->dim == 2) {
        const size_t byb = std::max<size_t>(1, kMbnkBatchDoubles / L.N);
        const size_t lim_grid = (size_t)65535 / L.nb;
        const size_t lim_idx = ((size_t)1 << 31) / ((size_t)m.Ne * std::max(m.n[0], m.n[1]) + 1);
        batch = (int)std::max<size_t>(1, std::min({byb, lim_grid, lim_idx, (size_t)mb->ncolour * L.nb}));
    }
    mb->batch = batch;
    const size_t ntr = (size_t)ctx->dim * ctx->nv * L.NF * m.Ne * batch;
    mb->qb = dalloc(ctx, L.N * batch);
    mb->rb = dalloc(ctx, L.N * batch);
    mb->Jpb = dalloc(ctx, ntr);
    mb->Fsb = dalloc(ctx, ntr);
    mb->mmax = kMbnkMaxIt;
    mb->V = dalloc(ctx, (size_t)(kMbnkMaxIt + 1) * L.N);
    mb->Z = dalloc(ctx, (size_t)kMbnkMaxIt * L.N);
    mb->w = dalloc(ctx, L.N);
    mb->gm = dalloc(ctx, kMbnkGm);
    void *p = nullptr;
    HIPCHK(hipMalloc(&p, sizeof(int)));
    mb->status = (int *)p;
    mb->allocated = true;
}

// Assemble sigma I - dR/dq of a level at dq on the face-neighbour block
// pattern and factor it by red-black block ILU0.
void mbnk_factor_impl(frpmg_ctx *ctx, int level, const double *dq, double sigma, hipStream_t s) {
    REQUIRE(level >= 0 && level < ctx->nlevels, "bad level");
    Level &L = ctx->lv[level];
    REQUIRE(!L.pa, "MBNK smoothing is not available on mixed-degree levels");
    REQUIRE(L.nb <= kMbnkMaxNb, "MBNK takes element blocks of at most 136 unknowns");
    for (int a = 0; a < ctx->dim; ++a)
        REQUIRE(ctx->mesh.n[a] >= 4 && ctx->mesh.n[a] % 2 == 0,
                "MBNK needs an even element count of at least 4 per axis (red-black order, distinct neighbours)");
    mbnk_alloc(ctx, level);
    ensure_face_save(ctx, L);
    Mbnk &mb = *ctx->mb;
    mb.ready = false;
    ctx->graph_epoch++;
    HIPCHK(hipMemsetAsync(mb.status, 0, sizeof(int), s));
    HIPCHK(launch_ej_form(ctx, level, dq, sigma, s, mb.D));  // diagonal blocks and L.r0 = R(dq)
    const int npairs = mb.ncolour * mb.nb;
    for (int p0 = 0; p0 < npairs; p0 += mb.batch) {
        const int cnt = std::min(mb.batch, npairs - p0);
        HIPCHK(mb_perturb(ctx, mb, dq, p0, cnt, s));
        HIPCHK(launch_residual_batch(ctx, level, cnt, mb.qb, mb.rb, mb.Jpb, mb.Fsb, s));
        HIPCHK(mb_extract(ctx, mb, dq, L.r0, p0, cnt, s));
    }
    HIPCHK(mb_gather_red(ctx, mb, s));
    HIPCHK(invert_blocks_f64(mb.Ne / 2, mb.nb, mb.Rinv, mb.Rinv, mb.status, s));
    HIPCHK(mb_schur(ctx, mb, s));
    HIPCHK(invert_blocks_f64(mb.Ne / 2, mb.nb, mb.Binv, mb.Binv, mb.status, s));
    int flag = 0;
    HIPCHK(hipMemcpyAsync(ctx->host_pinned, mb.status, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    std::memcpy(&flag, ctx->host_pinned, sizeof(int));
    if (flag & kPivNonfinite) {
        ctx->err = "non-finite pivot in an MBNK block (NaN or Inf in the blocks)";
        throw Fail{FR_ENONFINITE};
    }
    if (flag) {
        ctx->err = "zero pivot in an MBNK block";
        throw Fail{FR_ESINGULAR};
    }
    mb.ready = true;
}

const Mbnk &mbnk_of(frpmg_ctx *ctx, int level) {
    REQUIRE(ctx->mb && ctx->mb->ready && (level < 0 || ctx->mb->level == level),
            "no MBNK factorisation of the level (mbnk_factor)");
    return *ctx->mb;
}

// ---------------------------------------------------------------------------
// learned coarse correction: buffers, forward pass, training step
// ---------------------------------------------------------------------------

int round_up(int x, int m) { return (x + m - 1) / m * m; }

template <typename T>
T *talloc(frpmg_ctx *ctx, size_t n) {
    void *p = nullptr;
    HIPCHK(hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T)));
    return (T *)p;
}

void lcc_init_weights(frpmg_ctx *ctx, uint64_t seed) {
    Lcc &L = *ctx->lcc;
    std::mt19937_64 rng(seed);
    for (int l = 0; l < 3; ++l) {
        const int rows = L.wrows[l], cols = L.wcols[l];
        const int fan_in = (l == 0) ? L.nin : L.nh;
        const int live_rows = (l == 2) ? L.nout : rows;
        const int live_cols = (l == 0) ? L.nin : cols;
        const double sd = std::sqrt(2.0 / fan_in) * (l == 2 ? 0.5 : 1.0);
        std::normal_distribution<double> nd(0.0, sd);
        std::vector<float> w((size_t)rows * cols, 0.f);
        for (int r = 0; r < live_rows; ++r)
            for (int q = 0; q < live_cols; ++q) w[(size_t)r * cols + q] = (float)nd(rng);
        HIPCHK(hipMemcpy(L.W[l], w.data(), w.size() * sizeof(float), hipMemcpyHostToDevice));
        HIPCHK(hipMemset(L.Mo[l], 0, w.size() * sizeof(float)));
        HIPCHK(hipMemset(L.Vo[l], 0, w.size() * sizeof(float)));
        HIPCHK(lcc_to_bf(w.size(), L.W[l], L.Wb[l], nullptr));
    }
    L.adam_step = 0;
    HIPCHK(hipDeviceSynchronize());
}

void lcc_alloc(frpmg_ctx *ctx) {
    if (ctx->lcc) return;
    REQUIRE(ctx->nlevels > 1, "the learned correction needs two levels");
    REQUIRE(!ctx->lv[0].pa, "the learned correction is not available on mixed-degree levels");
    Lcc *Lp = new Lcc();
    ctx->lcc = Lp;
    Lcc &L = *Lp;
    const Level &C = ctx->lv[1];
    L.ngeo = ctx->dim;
    L.nin = C.nb * (1 + 2 * ctx->dim) + L.ngeo;
    L.nin_pad = round_up(L.nin, 32);
    L.nout = C.nb;
    L.nout_pad = round_up(L.nout, 32);
    L.wrows[0] = L.nh; L.wcols[0] = L.nin_pad;
    L.wrows[1] = L.nh; L.wcols[1] = L.nh;
    L.wrows[2] = L.nout_pad; L.wcols[2] = L.nh;
    for (int l = 0; l < 3; ++l) {
        const size_t n = (size_t)L.wrows[l] * L.wcols[l];
        L.W[l] = talloc<float>(ctx, n);
        L.G[l] = talloc<float>(ctx, n);
        L.Mo[l] = talloc<float>(ctx, n);
        L.Vo[l] = talloc<float>(ctx, n);
        L.Wb[l] = talloc<__bf16>(ctx, n);
        L.WbT[l] = talloc<__bf16>(ctx, n);
    }
    for (int a = 0; a < ctx->dim; ++a) {
        std::vector<double> ih(ctx->mesh.n[a]);
        HIPCHK(hipMemcpy(ih.data(), ctx->inv2h[a], ih.size() * sizeof(double), hipMemcpyDeviceToHost));
        double hm = 0.0;
        for (double x : ih) hm = std::max(hm, 2.0 / x);
        L.hmax[a] = hm;
    }
    L.in_scale = talloc<float>(ctx, 8);
    L.out_scale = talloc<float>(ctx, 8);
    const int Ne = ctx->mesh.Ne;
    L.Mpad = round_up(2 * Ne, 32);
    L.Xf = talloc<float>(ctx, (size_t)Ne * L.nin_pad);
    L.Tf = talloc<float>(ctx, (size_t)Ne * L.nout_pad);
    L.srow = talloc<float>(ctx, Ne);
    L.Xb = talloc<__bf16>(ctx, (size_t)L.Mpad * L.nin_pad);
    HIPCHK(hipMemset(L.Xb, 0, (size_t)L.Mpad * L.nin_pad * sizeof(__bf16)));
    L.H1 = talloc<__bf16>(ctx, (size_t)L.Mpad * L.nh);
    L.H2 = talloc<__bf16>(ctx, (size_t)L.Mpad * L.nh);
    L.Y = talloc<float>(ctx, (size_t)L.Mpad * L.nout_pad);
    L.dtmp = dalloc(ctx, C.N);
    L.Cuse = dalloc(ctx, C.N);
    L.lpart = dalloc(ctx, 64);
    L.lval = dalloc(ctx, 8);
    lcc_init_weights(ctx, 0x5eed1234ULL);
}

void lcc_free(frpmg_ctx *ctx) {
    if (!ctx->lcc) return;
    Lcc &L = *ctx->lcc;
    for (int l = 0; l < 3; ++l) {
        dfree(L.W[l]); dfree(L.G[l]); dfree(L.Mo[l]); dfree(L.Vo[l]); dfree(L.Wb[l]); dfree(L.WbT[l]);
    }
    void *bufs[] = {L.in_scale, L.out_scale, L.HX, L.HT, L.Xf, L.Tf, L.srow, L.Y, L.Xb, L.H1, L.H2, L.dtmp, L.Cuse,
                    L.bX, L.bXT, L.bH1, L.bH1T, L.bH2, L.bH2T, L.bdY, L.bdYT, L.bdH2, L.bdH2T, L.bdH1, L.bdH1T,
                    L.bY, L.bT, L.perm, L.lpart, L.lval};
    for (void *b : bufs) dfree(b);
    delete ctx->lcc;
    ctx->lcc = nullptr;
}

void lcc_train_buffers(frpmg_ctx *ctx, int B) {
    Lcc &L = *ctx->lcc;
    if (L.B == B) return;
    void *bufs[] = {L.bX, L.bXT, L.bH1, L.bH1T, L.bH2, L.bH2T, L.bdY, L.bdYT, L.bdH2, L.bdH2T, L.bdH1, L.bdH1T,
                    L.bY, L.bT};
    for (void *b : bufs) dfree(b);
    L.B = B;
    L.bX = talloc<__bf16>(ctx, (size_t)B * L.nin_pad);
    L.bXT = talloc<__bf16>(ctx, (size_t)B * L.nin_pad);
    L.bH1 = talloc<__bf16>(ctx, (size_t)B * L.nh);
    L.bH1T = talloc<__bf16>(ctx, (size_t)B * L.nh);
    L.bH2 = talloc<__bf16>(ctx, (size_t)B * L.nh);
    L.bH2T = talloc<__bf16>(ctx, (size_t)B * L.nh);
    L.bdY = talloc<__bf16>(ctx, (size_t)B * L.nout_pad);
    L.bdYT = talloc<__bf16>(ctx, (size_t)B * L.nout_pad);
    L.bdH2 = talloc<__bf16>(ctx, (size_t)B * L.nh);
    L.bdH2T = talloc<__bf16>(ctx, (size_t)B * L.nh);
    L.bdH1 = talloc<__bf16>(ctx, (size_t)B * L.nh);
    L.bdH1T = talloc<__bf16>(ctx, (size_t)B * L.nh);
    L.bY = talloc<float>(ctx, (size_t)B * L.nout_pad);
    L.bT = talloc<float>(ctx, (size_t)B * L.nout_pad);
}

// H1 = relu(X W1^T), H2 = relu(H1 W2^T), Y = H2 W3^T for M rows
void lcc_forward_rows(frpmg_ctx *ctx, int M, const __bf16 *X, __bf16 *H1, __bf16 *H2, float *Y, hipStream_t s) {
    Lcc &L = *ctx->lcc;
    HIPCHK(lcc_gemm(LCC_EP_RELU, M, L.nh, L.nin_pad, X, L.nin_pad, L.Wb[0], L.nin_pad, nullptr, H1, L.nh, nullptr,
                    1.f, s));
    HIPCHK(lcc_gemm(LCC_EP_RELU, M, L.nh, L.nh, H1, L.nh, L.Wb[1], L.nh, nullptr, H2, L.nh, nullptr, 1.f, s));
    HIPCHK(lcc_gemm(LCC_EP_F32, M, L.nout_pad, L.nh, H2, L.nh, L.Wb[2], L.nh, Y, nullptr, L.nout_pad, nullptr, 1.f,
                    s));
}

// loss and gradients of one batch already in L.bX / L.bT (B rows)
void lcc_batch_grad(frpmg_ctx *ctx, hipStream_t s) {
    Lcc &L = *ctx->lcc;
    const int B = L.B;
    lcc_forward_rows(ctx, B, L.bX, L.bH1, L.bH2, L.bY, s);
    HIPCHK(lcc_loss_grad(B, L.nout_pad, L.nout, L.bY, L.bT, L.bdY, L.lpart, L.lval, s));
    // dW3 = dY^T H2
    HIPCHK(lcc_transpose(B, L.nout_pad, L.bdY, L.nout_pad, L.bdYT, B, s));
    HIPCHK(lcc_transpose(B, L.nh, L.bH2, L.nh, L.bH2T, B, s));
    HIPCHK(lcc_gemm(LCC_EP_F32, L.nout_pad, L.nh, B, L.bdYT, B, L.bH2T, B, L.G[2], nullptr, L.nh, nullptr, 1.f, s));
    // dH2 = (dY W3) * [H2 > 0]
    HIPCHK(lcc_transpose(L.nout_pad, L.nh, L.Wb[2], L.nh, L.WbT[2], L.nout_pad, s));
    HIPCHK(lcc_gemm(LCC_EP_MASK, B, L.nh, L.nout_pad, L.bdY, L.nout_pad, L.WbT[2], L.nout_pad, nullptr, L.bdH2, L.nh,
                    L.bH2, 1.f, s));
    // dW2 = dH2^T H1
    HIPCHK(lcc_transpose(B, L.nh, L.bdH2, L.nh, L.bdH2T, B, s));
    HIPCHK(lcc_transpose(B, L.nh, L.bH1, L.nh, L.bH1T, B, s));
    HIPCHK(lcc_gemm(LCC_EP_F32, L.nh, L.nh, B, L.bdH2T, B, L.bH1T, B, L.G[1], nullptr, L.nh, nullptr, 1.f, s));
    // dH1 = (dH2 W2) * [H1 > 0]
    HIPCHK(lcc_transpose(L.nh, L.nh, L.Wb[1], L.nh, L.WbT[1], L.nh, s));
    HIPCHK(lcc_gemm(LCC_EP_MASK, B, L.nh, L.nh, L.bdH2, L.nh, L.WbT[1], L.nh, nullptr, L.bdH1, L.nh, L.bH1, 1.f, s));
    // dW1 = dH1^T X
    HIPCHK(lcc_transpose(B, L.nh, L.bdH1, L.nh, L.bdH1T, B, s));
    HIPCHK(lcc_transpose(B, L.nin_pad, L.bX, L.nin_pad, L.bXT, B, s));
    HIPCHK(lcc_gemm(LCC_EP_F32, L.nh, L.nin_pad, B, L.bdH1T, B, L.bXT, B, L.G[0], nullptr, L.nin_pad, nullptr, 1.f,
                    s));
}

// per-variable RMS of a level-1 field (host), 1 where the field vanishes
void lcc_rms(frpmg_ctx *ctx, const double *d, float *out) {
    const Level &C = ctx->lv[1];
    std::vector<double> h(C.N);
    HIPCHK(hipMemcpy(h.data(), d, C.N * sizeof(double), hipMemcpyDeviceToHost));
    const size_t per = (size_t)C.Np * ctx->mesh.Ne;
    for (int v = 0; v < ctx->nv; ++v) {
        double ss = 0.0;
        for (size_t i = 0; i < per; ++i) ss += h[v * per + i] * h[v * per + i];
        const double r = std::sqrt(ss / per);
        out[v] = (r > 0.0 && std::isfinite(r)) ? (float)r : 1.f;
    }
}

// ---------------------------------------------------------------------------
// nonlinear p-multigrid preconditioner
// ---------------------------------------------------------------------------

void pmg_point(frpmg_ctx *ctx, const double *dq, const double *rq, hipStream_t s) {
    ctx->pt_q = dq;
    ctx->pt_rq = rq;
    HIPCHK(vec_dot(ctx, ctx->lv[0].N, dq, dq, ctx->scal + SC_PT_N2, s));
    for (int l = 1; l < ctx->nlevels; ++l) {
        HIPCHK(transfer_apply(ctx, l - 1, true, l == 1 ? dq : ctx->mq[l - 1], ctx->mq[l], s));
        residual(ctx, l, ctx->mq[l], ctx->mr[l], s);
    }
}

int pmg_sweeps(const pmg_params &p, int l) {
    return l == 0 ? p.n0 : l == 1 ? p.n1 : l == 2 ? p.n2 : p.n3;
}

// Levels l >= 1 of the FAS V-cycle (Sec. 3.1 applied recursively).  On entry:
// Z0[l] = Gamma Y_{l-1}, cd[l] = Gamma G_{l-1}(Y_{l-1}) = -Gamma d_{l-1} and the
// forcing S[l] = G_l(Z0; 0) + Gamma d_{l-1}, so that G_l(Z0; S) = cd[l].  On exit
// Z[l] is the smoothed level-l solution.  G_l(Z; S) = sigma_D Z - [R_l(q_l + Z)
// - R_l(q_l)] - S.
void coarse_cycle(frpmg_ctx *ctx, const pmg_params &p, int l, int nlev, hipStream_t s, Counters *cnt) {
    const Scal one{1.0, nullptr};
    const int n = pmg_sweeps(p, l);
    REQUIRE(n >= 1, "every coarse level needs at least one sweep (n1, n2, n3 >= 1)");
    long &R = cnt->R1;  // every coarse level counts as coarse
    long &E = cnt->E1;
    double *Z0 = ctx->mZ0[l], *Z = ctx->mZ[l], *S = ctx->mS[l], *G = ctx->mG[l], *cd = ctx->md[l];
    if (p.coarse_mode == FR_COARSE_MBNK && l == nlev - 1) {
        // MBNK sweeps on the coarsest level: Z <- Z - (sigma_S I - J)^{-1} G_l(Z) by GMRES
        const Mbnk &mb = mbnk_of(ctx, l);
        const int maxit = p.mbnk_maxit > 0 ? p.mbnk_maxit : 5;
        const double tol = p.mbnk_tol > 0 ? p.mbnk_tol : 0.1;
        REQUIRE(maxit <= kMbnkMaxIt, "mbnk_maxit exceeds 8");
        HIPCHK(mb_sweep(ctx, mb, cd, Z0, Z, tol, maxit, s));
        E++;
        for (int it = 1; it < n; ++it) {
            residual_lin(ctx, l, ctx->mq[l], Z, one, ctx->mr[l], p.sigma_D, S, G, s);
            R++;
            HIPCHK(mb_sweep(ctx, mb, G, Z, Z, tol, maxit, s));
            E++;
        }
        return;
    }
    REQUIRE(ctx->lv[l].inv_prec >= 0, "a coarse level has no EJ factors");
    // the first sweep starts from Z0, where G_l = cd: Z = Z0 - B_l^{-1} cd
    HIPCHK(ej_apply_ex(ctx, l, cd, -1.0, 1.0, Z0, one, Z, s));
    E++;
    for (int it = 1; it < n; ++it) {
        residual_lin(ctx, l, ctx->mq[l], Z, one, ctx->mr[l], p.sigma_D, S, G, s);
        R++;
        HIPCHK(ej_apply(ctx, l, G, -1.0, 1.0, Z, s));
        E++;
    }
    if (l == nlev - 1) return;
    // defect, restriction and FAS forcing of level l + 1
    residual_lin(ctx, l, ctx->mq[l], Z, one, ctx->mr[l], p.sigma_D, S, G, s);
    R++;
    HIPCHK(transfer_restrict2(ctx, l, Z, ctx->mZ0[l + 1], G, ctx->md[l + 1], s));
    residual_lin(ctx, l + 1, ctx->mq[l + 1], ctx->mZ0[l + 1], one, ctx->mr[l + 1], p.sigma_D, ctx->md[l + 1],
                 ctx->mS[l + 1], s);
    cnt->R1++;
    coarse_cycle(ctx, p, l + 1, nlev, s, cnt);
    // Z += Pi (Z_{l+1} - Z0_{l+1}), then post-smoothing
    HIPCHK(transfer_apply(ctx, l, false, ctx->mZ[l + 1], Z, s, ctx->mZ0[l + 1], true));
    for (int it = 0; it < n; ++it) {
        residual_lin(ctx, l, ctx->mq[l], Z, one, ctx->mr[l], p.sigma_D, S, G, s);
        R++;
        HIPCHK(ej_apply(ctx, l, G, -1.0, 1.0, Z, s));
        E++;
    }
}

void pmg_apply_impl(frpmg_ctx *ctx, const pmg_params &p, const double *x, double *y, hipStream_t s,
                    Counters *cnt) {
    REQUIRE(ctx->pt_q && ctx->pt_rq, "pmg_set_point has not been called");
    REQUIRE(p.n0 >= 1, "n0 must be >= 1");
    const Level &L0 = ctx->lv[0];
    REQUIRE(L0.inv_prec >= 0, "level 0 has no EJ factors");
    const size_t N0 = L0.N;
    const bool coarse = p.coarse_mode != FR_COARSE_NONE;
    const bool learned = p.coarse_mode == FR_COARSE_LEARNED;
    const int nlev = learned ? 2 : (p.levels > 0 ? p.levels : ctx->nlevels);
    if (coarse) {
        REQUIRE(ctx->nlevels > 1, "pMG needs two levels");
        REQUIRE(nlev >= 2 && nlev <= ctx->nlevels, "the cycle's levels exceed the context's");
        if (learned) {
            REQUIRE(ctx->lcc && ctx->lcc->scales_set, "the learned correction has no trained network");
        } else {
            REQUIRE(p.coarse_mode == FR_COARSE_EJ || p.coarse_mode == FR_COARSE_MBNK, "unknown coarse mode");
            if (p.coarse_mode == FR_COARSE_MBNK) (void)mbnk_of(ctx, nlev - 1);
            else REQUIRE(ctx->lv[1].inv_prec >= 0, "level 1 has no EJ factors");
            REQUIRE(p.n1 >= 1, "n1 must be >= 1");
        }
    }
    const Scal one{1.0, nullptr};
    const double *Xs = x;
    Scal inv_s{1.0, nullptr};
    if (p.scale_mode == FR_SCALE_NORMALIZED || p.scale_mode == FR_SCALE_SCALED) {
        HIPCHK(vec_dot_pmg_scale(ctx, N0, x, p.scale_mode == FR_SCALE_SCALED ? ctx->scal + SC_PT_N2 : nullptr,
                                 p.eps_p, p.sigma_D, ctx->scal + SC_PMG_N2, ctx->scal + SC_PMG_S,
                                 ctx->scal + SC_PMG_INV, s));
        HIPCHK(vec_scale_copy(N0, Scal{0.0, ctx->scal + SC_PMG_S}, x, ctx->wXs, s));
        Xs = ctx->wXs;
        inv_s = Scal{0.0, ctx->scal + SC_PMG_INV};
    }
    double *Y = ctx->wY, *G = ctx->wG;
    // post-smoothing; the last sweep writes the output, undoing the input scale
    bool scaled_out = false;
    auto post_smooth = [&]() {
        for (int it = 0; it < p.n0; ++it) {
            residual_lin(ctx, 0, ctx->pt_q, Y, one, ctx->pt_rq, p.sigma_D, Xs, G, s);
            cnt->R0++;
            const bool last = it == p.n0 - 1;
            HIPCHK(ej_apply_ex(ctx, 0, G, -1.0, 1.0, Y, last ? inv_s : one, last ? y : Y, s));
            cnt->E0++;
        }
        scaled_out = true;
    };
    // pre-smoothing: the first sweep starts at Y = 0, where G = -X
    HIPCHK(ej_apply(ctx, 0, Xs, 1.0, 0.0, Y, s));
    cnt->E0++;
    for (int it = 1; it < p.n0; ++it) {
        residual_lin(ctx, 0, ctx->pt_q, Y, one, ctx->pt_rq, p.sigma_D, Xs, G, s);
        cnt->R0++;
        HIPCHK(ej_apply(ctx, 0, G, -1.0, 1.0, Y, s));
        cnt->E0++;
    }
    if (coarse && learned) {
        // defect d = -G(Y), restricted; the network maps Gamma d to the coarse correction
        Lcc &Lc = *ctx->lcc;
        const size_t N1 = ctx->lv[1].N;
        residual_lin(ctx, 0, ctx->pt_q, Y, one, ctx->pt_rq, p.sigma_D, Xs, G, s);
        cnt->R0++;
        HIPCHK(transfer_apply(ctx, 0, true, G, ctx->cd, s));
        // base: the element-local coarse EJ step C1 = B1^{-1} Gamma d
        HIPCHK(ej_apply(ctx, 1, ctx->cd, -1.0, 0.0, Lc.dtmp, s));
        cnt->E1++;
        HIPCHK(lcc_features(ctx, Lc.dtmp, Lc, Lc.Xf, Lc.Xb, Lc.srow, 1, s));
        lcc_forward_rows(ctx, Lc.Mpad, Lc.Xb, Lc.H1, Lc.H2, Lc.Y, s);
        HIPCHK(lcc_output(ctx, Lc, Lc.Y, Lc.srow, ctx->cZ, s));
        HIPCHK(vec_axpby(N1, one, Lc.dtmp, one, ctx->cZ, s));  // C = C1 + network refinement
        HIPCHK(transfer_apply(ctx, 0, false, ctx->cZ, Y, s, nullptr, true));  // Y += Pi C
        post_smooth();
    } else if (coarse) {
        const size_t N1 = ctx->lv[1].N;
        // defect d = -G(Y); restrict Y and G
        residual_lin(ctx, 0, ctx->pt_q, Y, one, ctx->pt_rq, p.sigma_D, Xs, G, s);
        cnt->R0++;
        HIPCHK(transfer_restrict2(ctx, 0, Y, ctx->cZ0, G, ctx->cd, s));  // cd = Gamma G = -Gamma d
        // FAS forcing S1 = G1(Z0) + Gamma d  with G1(Z) = sigma Z - (R1(q1 + Z) - R1(q1))
        residual_lin(ctx, 1, ctx->q1, ctx->cZ0, one, ctx->r1, p.sigma_D, ctx->cd, ctx->cS, s);
        cnt->R1++;
        // coarse levels (recursively below level 1); the first level-1 sweep uses
        // G1(Z0) - S1 = -Gamma d = cd
        coarse_cycle(ctx, p, 1, nlev, s, cnt);
        if (nlev == 2 && ctx->lcc && ctx->lcc->harvesting && ctx->lcc->count < ctx->lcc->cap) {
            // record (Gamma d, correction after target_sweeps coarse sweeps) for a rotating subset
            Lcc &Lc = *ctx->lcc;
            HIPCHK(hipMemcpyAsync(Lc.Cuse, ctx->cZ, N1 * sizeof(double), hipMemcpyDeviceToDevice, s));
            for (int it = p.n1; it < Lc.target_sweeps; ++it) {
                residual_lin(ctx, 1, ctx->q1, ctx->cZ, one, ctx->r1, p.sigma_D, ctx->cS, ctx->cG, s);
                HIPCHK(ej_apply(ctx, 1, ctx->cG, -1.0, 1.0, ctx->cZ, s));
            }
            HIPCHK(vec_axpby(N1, Scal{-1.0, nullptr}, ctx->cZ0, Scal{1.0, nullptr}, ctx->cZ, s));  // target C
            // network input: the element-local first sweep C1 = B1^{-1} Gamma d;
            // network target: what the deeper coarse solve adds to it
            HIPCHK(ej_apply(ctx, 1, ctx->cd, -1.0, 0.0, Lc.dtmp, s));
            HIPCHK(vec_axpby(N1, Scal{-1.0, nullptr}, Lc.dtmp, Scal{1.0, nullptr}, ctx->cZ, s));
            if (!Lc.scales_set) {
                HIPCHK(hipStreamSynchronize(s));
                lcc_rms(ctx, Lc.dtmp, Lc.h_in_scale);
                lcc_rms(ctx, ctx->cZ, Lc.h_out_scale);
                HIPCHK(hipMemcpy(Lc.in_scale, Lc.h_in_scale, 5 * sizeof(float), hipMemcpyHostToDevice));
                HIPCHK(hipMemcpy(Lc.out_scale, Lc.h_out_scale, 5 * sizeof(float), hipMemcpyHostToDevice));
                Lc.scales_set = 1;
            }
            HIPCHK(lcc_features(ctx, Lc.dtmp, Lc, Lc.Xf, Lc.Xb, Lc.srow, 0, s));
            HIPCHK(lcc_targets(ctx, ctx->cZ, Lc, Lc.srow, Lc.Tf, s));
            const int Ne = ctx->mesh.Ne;
            const int offset = Lc.cycle % Lc.stride;
            const int nsel = (Ne - offset + Lc.stride - 1) / Lc.stride;
            HIPCHK(lcc_harvest_rows(Lc, Ne, Lc.stride, offset, Lc.count, Lc.Xf, Lc.Tf, s));
            Lc.count = std::min(Lc.cap, Lc.count + nsel);
            Lc.cycle++;
            HIPCHK(hipMemcpyAsync(ctx->cZ, Lc.Cuse, N1 * sizeof(double), hipMemcpyDeviceToDevice, s));
        }
        // Y += Pi (Z - Z0), one kernel
        HIPCHK(transfer_apply(ctx, 0, false, ctx->cZ, Y, s, ctx->cZ0, true));
        post_smooth();
    }
    if (!scaled_out) HIPCHK(vec_scale_copy(N0, inv_s, Y, y, s));
}

// ---------------------------------------------------------------------------
// flexible GMRES(m)
// ---------------------------------------------------------------------------

struct KrylovResult {
    int iters = 0, restarts = 0;
    bool converged = false, breakdown = false, nonfinite = false, restarted_nonfinite = false;
    double res_est = 0.0, bnorm = 0.0;
    double true_res = -1.0;  // ||b - A x|| recomputed at the end (verify), else -1
};

// Stall monitor: when the residual estimate fails to drop below ratio times
// its value window iterations earlier, on_stall() is called once.
struct Stall {
    bool active = false;
    int window = 5;
    double ratio = 0.7;
    std::vector<double> hist;
    std::function<void()> on_stall;
};

void clear_graphs(frpmg_ctx *ctx) {
    for (auto &g : ctx->graphs)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    ctx->graphs.clear();
}

// Launch the captured graph of `body` for this key on s, capturing and
// instantiating it on first use (on the context's capture stream, so nothing
// runs while it is recorded).  cnt receives the operation counts of one
// replay.
template <typename Body>
void run_graph(frpmg_ctx *ctx, const std::vector<unsigned long long> &key, Counters *cnt, Body &&body,
               hipStream_t s) {
    for (const auto &g : ctx->graphs) {
        if (g.key == key) {
            HIPCHK(hipGraphLaunch(g.exec, s));
            cnt->R0 += g.dR0;
            cnt->R1 += g.dR1;
            cnt->E0 += g.dE0;
            cnt->E1 += g.dE1;
            return;
        }
    }
    if (ctx->graphs.size() >= 256) clear_graphs(ctx);
    if (!ctx->cap_stream) HIPCHK(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
    const Counters before = *cnt;
    HIPCHK(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
    try {
        body(ctx->cap_stream);
    } catch (...) {
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(ctx->cap_stream, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
    }
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamEndCapture(ctx->cap_stream, &g));
    hipGraphExec_t ex = nullptr;
    const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HIPCHK(e);
    StepGraph sg;
    sg.key = key;
    sg.exec = ex;
    sg.dR0 = cnt->R0 - before.R0;
    sg.dR1 = cnt->R1 - before.R1;
    sg.dE0 = cnt->E0 - before.E0;
    sg.dE1 = cnt->E1 - before.E1;
    ctx->graphs.push_back(std::move(sg));
    HIPCHK(hipGraphLaunch(ex, s));
}

// What a captured Arnoldi step depends on besides its index: null when the
// steps are launched from the host.
struct GraphUse {
    std::vector<unsigned long long> key;
    Counters *cnt = nullptr;
};

unsigned long long bits(double v) {
    unsigned long long u;
    std::memcpy(&u, &v, sizeof(u));
    return u;
}
unsigned long long bits(const void *p) { return (unsigned long long)(uintptr_t)p; }

template <typename MatVec, typename Prec>
KrylovResult fgmres(frpmg_ctx *ctx, size_t N, const double *b, double *x, int m, double tol, int max_restarts,
                    MatVec &&A, Prec &&M, hipStream_t s, Stall *stall = nullptr, const GraphUse *gu = nullptr,
                    bool verify = false) {
    KrylovResult kr;
    double *V = ctx->V, *Z = ctx->Zk, *w = ctx->kw;
    const size_t ld = N;
    std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), yv(m);
    auto Hc = [&](int i, int j) -> double & { return H[(size_t)j * (m + 1) + i]; };
    HIPCHK(vec_fill(N, 0.0, x, s));
    const double bnorm = host_norm(ctx, N, b, s);
    kr.bnorm = bnorm;
    if (!std::isfinite(bnorm)) {
        kr.nonfinite = true;
        return kr;
    }
    if (bnorm == 0.0) {
        kr.converged = true;
        return kr;
    }
    const double target = tol * bnorm;
    double beta = bnorm;
    if (stall) {
        stall->hist.clear();
        stall->hist.push_back(bnorm);
    }
    HIPCHK(vec_scale_copy(N, Scal{1.0 / beta, nullptr}, b, V, s));
    for (;;) {
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int jend = 0;
        // Arnoldi step j (z_j = M v_j, w = A z_j, CGS2 against v_0..v_j,
        // v_{j+1} = w / ||w||, the norm kept on the device), then the copy of
        // its Hessenberg column to pinned buffer j & 1.  Step j + 1 needs only
        // v_{j+1}, so while the residual estimate is far from the target it
        // is enqueued before the host waits for step j: the GPU does not idle
        // for the host's round trip (64x64 p = 4: ~30 us per iteration).  A
        // step launched ahead of the one that converges is wasted work, so
        // near the target, and with the learned preconditioner (whose stall
        // fallback switches preconditioners between steps), steps run one at
        // a time.
        const bool timed = !gu && ctx->ph_ev[0];
        auto launch = [&](int jj) {
            const int buf = jj & 1;
            hipEvent_t *ev = ctx->ph_ev + 4 * buf;
            auto step = [&, jj, ev](hipStream_t st) {
                double *vj = V + (size_t)jj * ld;
                double *zj = Z + (size_t)jj * ld;
                if (timed) HIPCHK(hipEventRecord(ev[0], st));
                M(vj, zj, st);
                if (timed) HIPCHK(hipEventRecord(ev[1], st));
                A(zj, w, st);
                if (timed) HIPCHK(hipEventRecord(ev[2], st));
                HIPCHK(vec_mdot(ctx, N, jj + 1, V, ld, w, ctx->red_out + RO_H1, st));
                HIPCHK(vec_gemv_sub_mdot(ctx, N, jj + 1, V, ld, ctx->red_out + RO_H1, w, ctx->red_out + RO_H2, st));
                HIPCHK(vec_gemv_sub(N, jj + 1, V, ld, ctx->red_out + RO_H2, w, st));
                HIPCHK(vec_dot_normalize(ctx, N, w, ctx->red_out + RO_N2, V + (size_t)(jj + 1) * ld, st));
                if (timed) HIPCHK(hipEventRecord(ev[3], st));
            };
            if (gu) {
                std::vector<unsigned long long> key = gu->key;
                key.push_back((unsigned long long)jj);
                run_graph(ctx, key, gu->cnt, step, s);
            } else {
                Range r("arnoldi step");
                step(s);
            }
            // the Hessenberg column only (the y staging at RO_Y stays untouched)
            HIPCHK(hipMemcpyAsync(buf ? ctx->host_pinned2 : ctx->host_pinned, ctx->red_out,
                                  (RO_N2 + 1) * sizeof(double), hipMemcpyDeviceToHost, s));
            HIPCHK(hipEventRecord(ctx->step_ev[buf], s));
        };
        int launched = -1;         // the last step enqueued in this cycle
        double est = beta;         // the residual estimate before step j
        constexpr double kAhead = 30.0;  // launch ahead while the estimate exceeds kAhead x the target
        for (int j = 0; j < m; ++j) {
            if (launched < j) {
                launch(j);
                launched = j;
            }
            if (!stall && j + 1 < m && est > kAhead * target) {
                launch(j + 1);
                launched = j + 1;
            }
            HIPCHK(hipEventSynchronize(ctx->step_ev[j & 1]));
            if (timed) {
                for (int ph = 0; ph < 3; ++ph) {
                    float ms = 0.f;
                    HIPCHK(hipEventElapsedTime(&ms, ctx->ph_ev[4 * (j & 1) + ph], ctx->ph_ev[4 * (j & 1) + ph + 1]));
                    ctx->ph_acc[ph] += 1e-3 * ms;
                }
            }
            const double *hp = (j & 1) ? ctx->host_pinned2 : ctx->host_pinned;
            for (int i = 0; i <= j; ++i) Hc(i, j) = hp[RO_H1 + i] + hp[RO_H2 + i];
            const double hn = std::sqrt(hp[RO_N2]);
            Hc(j + 1, j) = hn;
            for (int i = 0; i < j; ++i) {
                const double t = cs[i] * Hc(i, j) + sn[i] * Hc(i + 1, j);
                Hc(i + 1, j) = -sn[i] * Hc(i, j) + cs[i] * Hc(i + 1, j);
                Hc(i, j) = t;
            }
            const double den = std::hypot(Hc(j, j), Hc(j + 1, j));
            cs[j] = Hc(j, j) / den;
            sn[j] = Hc(j + 1, j) / den;
            Hc(j, j) = den;
            Hc(j + 1, j) = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            kr.iters++;
            jend = j + 1;
            kr.res_est = std::fabs(g[j + 1]);
            est = kr.res_est;
            if (!std::isfinite(kr.res_est) || !std::isfinite(hn)) {
                if (stall && stall->active) {
                    // the learned preconditioner produced a non-finite direction:
                    // fall back and restart the cycle from the last iterate
                    stall->active = false;
                    stall->on_stall();
                    jend = 0;
                    kr.restarted_nonfinite = true;
                    break;
                }
                kr.nonfinite = true;
                return kr;
            }
            if (stall && stall->active) {
                stall->hist.push_back(kr.res_est);
                const size_t n = stall->hist.size();
                if ((int)n > stall->window && kr.res_est > stall->ratio * stall->hist[n - 1 - stall->window]) {
                    stall->active = false;
                    stall->on_stall();
                }
            }
            if (hn == 0.0) {
                kr.breakdown = true;
                break;
            }
            if (kr.res_est <= target) break;
        }
        if (kr.restarted_nonfinite) {
            // discard the cycle; restart from x with the true residual
            kr.restarted_nonfinite = false;
            kr.restarts++;
            A(x, w, s);
            HIPCHK(vec_axpby(N, Scal{1.0, nullptr}, b, Scal{-1.0, nullptr}, w, s));
            beta = host_norm(ctx, N, w, s);
            if (!std::isfinite(beta)) {
                kr.nonfinite = true;
                return kr;
            }
            kr.res_est = beta;
            if (beta <= target) {
                kr.converged = true;
                return kr;
            }
            HIPCHK(vec_scale_copy(N, Scal{1.0 / beta, nullptr}, w, V, s));
            continue;
        }
        // a step launched ahead of the one that ended the cycle finishes
        // first (it leaves x, and the basis the update uses, untouched)
        if (launched >= jend) HIPCHK(hipStreamSynchronize(s));
        // back substitution with the triangular Hessenberg factor
        for (int i = jend - 1; i >= 0; --i) {
            double t = g[i];
            for (int k = i + 1; k < jend; ++k) t -= Hc(i, k) * yv[k];
            yv[i] = t / Hc(i, i);
        }
        std::memcpy(ctx->host_pinned + RO_Y, yv.data(), jend * sizeof(double));
        HIPCHK(hipMemcpyAsync(ctx->red_out + RO_Y, ctx->host_pinned + RO_Y, jend * sizeof(double),
                              hipMemcpyHostToDevice, s));
        HIPCHK(vec_combine(N, jend, Z, ld, ctx->red_out + RO_Y, x, s));
        HIPCHK(hipStreamSynchronize(s));  // the pinned staging is reused below
        const bool est_done = kr.res_est <= target || kr.breakdown;
        const double prev_true = kr.true_res;
        if (est_done && (!verify || kr.breakdown)) {
            kr.converged = true;
            return kr;
        }
        // the cycle ran out, or (verify) its estimate met the tolerance: the
        // true residual r = b - A x decides, and a new cycle starts from it
        if (!est_done) {
            if (kr.restarts >= max_restarts) return kr;
            kr.restarts++;
        }
        A(x, w, s);
        HIPCHK(vec_axpby(N, Scal{1.0, nullptr}, b, Scal{-1.0, nullptr}, w, s));
        beta = host_norm(ctx, N, w, s);
        kr.res_est = beta;
        if (verify) kr.true_res = beta;
        if (!std::isfinite(beta)) {
            kr.nonfinite = true;
            return kr;
        }
        if (beta <= target) {
            kr.converged = true;
            return kr;
        }
        if (est_done) {
            // a further cycle only while the recomputed residual keeps falling;
            // once it stops (the floor of an FD operator: its truncation and
            // rounding), the estimate having met the tolerance, the solve ends
            // there and true_res reports the floor
            if (prev_true >= 0.0 && beta > 0.5 * prev_true) {
                kr.converged = true;
                return kr;
            }
            if (kr.restarts >= max_restarts) return kr;
            kr.restarts++;
        }
        HIPCHK(vec_scale_copy(N, Scal{1.0 / beta, nullptr}, w, V, s));
    }
}

void ensure_krylov(frpmg_ctx *ctx, int m) {
    const size_t N = ctx->lv[0].N;
    if (ctx->kdim >= m && ctx->V) return;
    dfree(ctx->V);
    dfree(ctx->Zk);
    ctx->V = nullptr;
    ctx->Zk = nullptr;
    ctx->V = dalloc(ctx, (size_t)(m + 1) * N);
    ctx->Zk = dalloc(ctx, (size_t)m * N);
    ctx->kdim = m;
    if (!ctx->kw) ctx->kw = dalloc(ctx, N);
    if (!ctx->sq) ctx->sq = dalloc(ctx, N);
    if (!ctx->srq) ctx->srq = dalloc(ctx, N);
    if (!ctx->sF) ctx->sF = dalloc(ctx, N);
    if (!ctx->sb) ctx->sb = dalloc(ctx, N);
    if (!ctx->sdx) ctx->sdx = dalloc(ctx, N);
    for (auto &e : ctx->ph_ev)
        if (!e) HIPCHK(hipEventCreate(&e));
    for (auto &e : ctx->step_ev)
        if (!e) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
}

double now() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}


// The solver state of one implicit stage: shifts, preconditioner settings,
// counters, the stall monitor and the graph keys.  One object serves every
// stage of a time step (same diagonal coefficient, same EJ factors).
struct StageSolver {
    frpmg_ctx *ctx;
    stage_params P;
    size_t N;
    bool esdirk, pmg, learned, use_graphs, nonlinear_pmg, mbnk;
    int nlev;
    double sigma_A, sigma_S;
    pmg_params pp;
    Counters cnt;
    Stall stall;
    int fallbacks = 0;

    StageSolver(frpmg_ctx *c, const stage_params &prm) : ctx(c), P(prm) {
        REQUIRE(P.scheme == FR_SCHEME_ESDIRK || P.scheme == FR_SCHEME_ROW, "bad scheme");
        REQUIRE(P.m >= 1 && P.m <= kMaxKdim, "Krylov dimension must be in 1..120");
        REQUIRE(valid_eps_mode(P.eps_mode), "bad eps_mode");
        REQUIRE(P.dt > 0 && P.a_ii > 0, "dt and a_ii must be positive");
        REQUIRE(P.precond >= FR_PRECOND_EJ && P.precond <= FR_PRECOND_PMG_LEARNED, "unknown preconditioner");
        pmg = P.precond != FR_PRECOND_EJ;
        learned = P.precond == FR_PRECOND_PMG_LEARNED;
        if (learned) REQUIRE(ctx->lcc && ctx->lcc->scales_set, "the learned correction has no trained network");
        REQUIRE(!pmg || ctx->nlevels > 1, "pMG needs two levels");
        N = ctx->lv[0].N;
        ensure_krylov(ctx, P.m);
        esdirk = P.scheme == FR_SCHEME_ESDIRK;
        REQUIRE(P.solver == FR_SOLVER_JFNK || P.solver == FR_SOLVER_PMG, "unknown solver");
        nonlinear_pmg = P.solver == FR_SOLVER_PMG;
        REQUIRE(!nonlinear_pmg || (esdirk && pmg && !learned), "the pMG nonlinear solver takes ESDIRK stages "
                                                               "with the plain pMG hierarchy");
        const double dtau = (P.dtau > 0) ? P.dtau : P.dt;
        // shifts: sigma_A of the outer operator, sigma_S of the smoother blocks; the pMG
        // nonlinear solver's cycles target the stage equation itself (no outer pseudo-time)
        sigma_A = (esdirk && !nonlinear_pmg) ? 1.0 / dtau + 1.0 / (P.a_ii * P.dt) : 1.0 / (P.a_ii * P.dt);
        sigma_S = 1.0 / dtau + sigma_A;
        nlev = pmg ? (learned ? 2 : (P.pmg_levels > 0 ? P.pmg_levels : ctx->nlevels)) : 1;
        REQUIRE(nlev <= ctx->nlevels, "pmg_levels exceeds the context's levels");
        REQUIRE(P.coarse_smoother == FR_SMOOTHER_EJ || P.coarse_smoother == FR_SMOOTHER_MBNK,
                "unknown coarse smoother");
        mbnk = pmg && P.coarse_smoother == FR_SMOOTHER_MBNK;
        REQUIRE(!mbnk || !learned, "the MBNK smoother takes the plain pMG hierarchy");
        REQUIRE(P.mbnk_maxit >= 0 && P.mbnk_maxit <= kMbnkMaxIt, "mbnk_maxit must be in 0..8");
        REQUIRE(P.smoother_refresh >= 0, "smoother_refresh must be >= 0");
        pp = pmg_params{sigma_A, P.n0, P.n1, learned ? FR_COARSE_LEARNED : (mbnk ? FR_COARSE_MBNK : FR_COARSE_EJ),
                        nonlinear_pmg ? FR_SCALE_LITERAL : P.scale_mode, P.eps_p, P.n2, P.n3, nlev,
                        P.mbnk_maxit, P.mbnk_tol};
        stall.active = learned;
        if (P.stall_window > 0) stall.window = P.stall_window;
        if (P.stall_ratio > 0) stall.ratio = P.stall_ratio;
        stall.on_stall = [this] {
            pp.coarse_mode = FR_COARSE_EJ;  // plain pMG for the rest of the stage
            fallbacks++;
        };
        use_graphs = P.graphs && !learned && !(ctx->lcc && ctx->lcc->harvesting);
    }

    // EJ factors at q^n (Sec. 2.2: once per physical time step)
    void setup(const double *dq_n, hipStream_t s) {
        if (pmg) {
            ej_factor_impl(ctx, 0, dq_n, sigma_S, P.precision, s);
            // the coarse blocks are linearised at the restricted q^n
            for (int l = 1; l < nlev; ++l) {
                HIPCHK(transfer_apply(ctx, l - 1, true, l == 1 ? dq_n : ctx->mq[l - 1], ctx->mq[l], s));
                if (mbnk && l == nlev - 1) {
                    // the coarsest level smooths with MBNK: its assembled operator instead of EJ blocks
                    mbnk_factor_impl(ctx, l, ctx->mq[l], sigma_S, s);
                    cnt.R1 += 1 + ctx->lv[l].nb * (1 + ctx->mb->ncolour);
                } else {
                    ej_factor_impl(ctx, l, ctx->mq[l], sigma_S, P.precision, s);
                    cnt.R1 += 1 + ctx->lv[l].nb;
                }
            }
        } else {
            ej_factor_impl(ctx, 0, dq_n, sigma_A, P.precision, s);
        }
        // one base evaluation plus the element-local columns (nb evaluations' worth)
        cnt.R0 += 1 + ctx->lv[0].nb;
    }

    // pMG as the nonlinear solver of an ESDIRK stage: V-cycles on F(q + Y) = 0
    fr_status pmg_nonlinear_solve(const double *b, double *q, double *rq, stage_stats *st, hipStream_t s) {
        double *F = ctx->sF, *dx = ctx->sdx;
        const double c = 1.0 / (P.a_ii * P.dt);
        HIPCHK(vec_stage_F(N, q, b, c, rq, F, s));
        const double f0 = host_norm(ctx, N, F, s);
        st->res0 = f0;
        double fn = f0;
        fr_status status = std::isfinite(f0) ? FR_OK : FR_ENONFINITE;
        while (status == FR_OK && fn > P.tol * f0 && st->ptc_iters < P.max_ptc) {
            if (P.smoother_refresh > 0 && st->ptc_iters > 0 && st->ptc_iters % P.smoother_refresh == 0)
                setup(q, s);  // smoothers re-formed at the current iterate
            pmg_point(ctx, q, rq, s);
            cnt.R1 += nlev - 1;
            HIPCHK(vec_axpby(N, Scal{0.0, nullptr}, nullptr, Scal{-1.0, nullptr}, F, s));  // F <- -F
            pmg_apply_impl(ctx, pp, F, dx, s, &cnt);
            HIPCHK(vec_axpby(N, Scal{1.0, nullptr}, dx, Scal{1.0, nullptr}, q, s));
            residual(ctx, 0, q, rq, s);
            cnt.R0++;
            HIPCHK(vec_stage_F(N, q, b, c, rq, F, s));
            fn = host_norm(ctx, N, F, s);
            st->ptc_iters++;
            if (!std::isfinite(fn)) status = FR_ENONFINITE;
        }
        st->res = fn;
        st->rel_res = f0 > 0 ? fn / f0 : 0.0;
        st->converged = (fn <= P.tol * f0) ? 1 : 0;
        if (status == FR_OK && !st->converged) status = FR_ENOCONV;
        return status;
    }

    void prec(const double *v, double *z, hipStream_t s) {
        if (pmg) {
            pmg_apply_impl(ctx, pp, v, z, s, &cnt);
        } else {
            HIPCHK(ej_apply(ctx, 0, v, 1.0, 0.0, z, s));
            cnt.E0++;
        }
    }

    // captured Arnoldi steps: everything a step bakes in goes into its key
    GraphUse graph_use(const double *q, const double *rq) {
        GraphUse g;
        g.cnt = &cnt;
        g.key = {ctx->graph_epoch, (unsigned long long)P.scheme, (unsigned long long)P.precond, bits(sigma_A),
                 bits(P.eps), (unsigned long long)P.eps_mode, (unsigned long long)P.n0, (unsigned long long)P.n1,
                 (unsigned long long)P.scale_mode, bits(P.eps_p), bits(q), bits(rq), bits(ctx->V), bits(ctx->Zk),
                 bits(ctx->kw), (unsigned long long)N, (unsigned long long)P.n2, (unsigned long long)P.n3,
                 (unsigned long long)nlev, (unsigned long long)pp.coarse_mode, (unsigned long long)P.mbnk_maxit,
                 bits(P.mbnk_tol)};
        return g;
    }

    // ESDIRK stage (Sec. 2.1 Eq. (ESDIRK2) and Sec. 2.2): F(q) = (q - b)/(a_ii dt)
    // - R(q) = 0 by pseudo-transient continuation with inexact Newton from q
    // (in/out, rq = R(q) in/out) until ||F|| <= tol ||F(q_start)||.
    fr_status esdirk_solve(const double *b, double *q, double *rq, stage_stats *st, hipStream_t s) {
        if (nonlinear_pmg) return pmg_nonlinear_solve(b, q, rq, st, s);
        double *F = ctx->sF, *dx = ctx->sdx;
        const double c = 1.0 / (P.a_ii * P.dt);
        HIPCHK(vec_stage_F(N, q, b, c, rq, F, s));
        const double f0 = host_norm(ctx, N, F, s);
        st->res0 = f0;
        double fn = f0;
        fr_status status = std::isfinite(f0) ? FR_OK : FR_ENONFINITE;
        auto prec_f = [&](const double *v, double *z, hipStream_t st2) { prec(v, z, st2); };
        while (status == FR_OK && fn > P.tol * f0 && st->ptc_iters < P.max_ptc) {
            if (pmg) {
                pmg_point(ctx, q, rq, s);
                cnt.R1 += ctx->nlevels - 1;
            }
            HIPCHK(vec_axpby(N, Scal{0.0, nullptr}, nullptr, Scal{-1.0, nullptr}, F, s));  // F <- -F
            HIPCHK(vec_dot(ctx, N, q, q, ctx->scal + SC_DQ_N2, s));
            auto A = [&](const double *z, double *w, hipStream_t st2) {
                jvp(ctx, 0, q, rq, z, sigma_A, P.eps, P.eps_mode, w, st2, ctx->scal + SC_DQ_N2);
                cnt.R0++;
            };
            const GraphUse gu = graph_use(q, rq);
            KrylovResult kr = fgmres(ctx, N, F, dx, P.m, P.eta, P.max_restarts, A, prec_f, s, &stall,
                                     use_graphs ? &gu : nullptr);
            if (st->ptc_iters < FR_MAX_NEWTON_LOG) st->gmres_per_newton[st->ptc_iters] = kr.iters;
            st->gmres_iters += kr.iters;
            st->restarts += kr.restarts;
            if (kr.nonfinite) {
                status = FR_ENONFINITE;
                break;
            }
            HIPCHK(vec_axpby(N, Scal{1.0, nullptr}, dx, Scal{1.0, nullptr}, q, s));
            residual(ctx, 0, q, rq, s);
            cnt.R0++;
            HIPCHK(vec_stage_F(N, q, b, c, rq, F, s));
            fn = host_norm(ctx, N, F, s);
            st->ptc_iters++;
            if (!std::isfinite(fn)) status = FR_ENONFINITE;
        }
        st->res = fn;
        st->rel_res = f0 > 0 ? fn / f0 : 0.0;
        st->converged = (fn <= P.tol * f0) ? 1 : 0;
        if (status == FR_OK && !st->converged) status = FR_ENOCONV;
        return status;
    }

    // ROW stage (Sec. 2.1 Eq. (Rosenbrock_General)): (sigma_A I - J(q_lin)) U = rhs
    // by FGMRES to tol relative to ||rhs||, J the FD Jacobian at q_lin (with
    // R_lin = R(q_lin)); the pMG point must already be at q_lin.
    fr_status row_solve(const double *q_lin, const double *R_lin, const double *rhs, double *U, stage_stats *st,
                        hipStream_t s) {
        double *w = ctx->sF;
        HIPCHK(vec_dot(ctx, N, q_lin, q_lin, ctx->scal + SC_DQ_N2, s));
        auto A = [&](const double *z, double *wout, hipStream_t st2) {
            jvp(ctx, 0, q_lin, R_lin, z, sigma_A, P.eps, P.eps_mode, wout, st2, ctx->scal + SC_DQ_N2);
            cnt.R0++;
        };
        auto prec_f = [&](const double *v, double *z, hipStream_t st2) { prec(v, z, st2); };
        const GraphUse gu = graph_use(q_lin, R_lin);
        // verify: the stage is solved when the recomputed residual of the FD
        // operator, not only the Krylov estimate, meets the tolerance
        KrylovResult kr = fgmres(ctx, N, rhs, U, P.m, P.tol, P.max_restarts, A, prec_f, s, &stall,
                                 use_graphs ? &gu : nullptr, P.verify != 0);
        st->gmres_iters += kr.iters;
        st->restarts += kr.restarts;
        st->gmres_per_newton[0] = kr.iters;
        st->res0 = kr.bnorm;
        st->res = kr.res_est;
        st->rel_res = kr.bnorm > 0 ? kr.res_est / kr.bnorm : 0.0;
        st->converged = kr.converged ? 1 : 0;
        // true residual of the FD operator at the solution
        double tr = kr.true_res;
        if (tr < 0.0) {
            A(U, w, s);
            HIPCHK(vec_axpby(N, Scal{1.0, nullptr}, rhs, Scal{-1.0, nullptr}, w, s));
            tr = host_norm(ctx, N, w, s);
        }
        st->true_rel_res = kr.bnorm > 0 ? tr / kr.bnorm : 0.0;
        if (kr.nonfinite) return FR_ENONFINITE;
        if (!kr.converged) return FR_ENOCONV;
        return FR_OK;
    }

    void finish(stage_stats *st) {
        st->n_R_fine = cnt.R0;
        st->n_R_coarse = cnt.R1;
        st->n_ej_fine = cnt.E0;
        st->n_ej_coarse = cnt.E1;
        st->fallbacks = fallbacks;
        st->t_precond = ctx->ph_acc[0];
        st->t_jvp = ctx->ph_acc[1];
        st->t_ortho = ctx->ph_acc[2];
    }
};

[[noreturn]] void fail_stage(frpmg_ctx *ctx, fr_status status) {
    ctx->err = status == FR_ENONFINITE ? "non-finite norm in the stage solve" : "stage solve did not converge";
    throw Fail{status};
}

void stage_impl(frpmg_ctx *ctx, const stage_params &P, const double *dq_n, double *out, stage_stats *st,
                hipStream_t s) {
    std::memset(st, 0, sizeof(*st));
    Range range("stage");
    StageSolver S(ctx, P);
    const size_t N = S.N;
    for (double &a : ctx->ph_acc) a = 0.0;
    HIPCHK(hipStreamSynchronize(s));
    const double t0 = now();
    if (!P.skip_setup) {
        Range rs("stage set-up");
        S.setup(dq_n, s);
    }
    HIPCHK(hipStreamSynchronize(s));
    const double t1 = now();
    fr_status status;
    if (S.esdirk) {
        // second stage of an ESDIRK scheme: b = q^n + dt a_i1 R(q^n), start at q^n
        double *q = ctx->sq, *rq = ctx->srq, *b = ctx->sb;
        residual(ctx, 0, dq_n, rq, s);
        S.cnt.R0++;
        HIPCHK(hipMemcpyAsync(b, dq_n, N * sizeof(double), hipMemcpyDeviceToDevice, s));
        HIPCHK(vec_axpby(N, Scal{P.a_i1 * P.dt, nullptr}, rq, Scal{1.0, nullptr}, b, s));
        HIPCHK(hipMemcpyAsync(q, dq_n, N * sizeof(double), hipMemcpyDeviceToDevice, s));
        status = S.esdirk_solve(b, q, rq, st, s);
        HIPCHK(hipMemcpyAsync(out, q, N * sizeof(double), hipMemcpyDeviceToDevice, s));
    } else {
        // first stage of a ROW scheme: rhs = R(q^n)
        double *R0 = ctx->srq;
        residual(ctx, 0, dq_n, R0, s);
        S.cnt.R0++;
        if (S.pmg) {
            pmg_point(ctx, dq_n, R0, s);
            S.cnt.R1 += ctx->nlevels - 1;
        }
        status = S.row_solve(dq_n, R0, R0, out, st, s);
    }
    HIPCHK(hipStreamSynchronize(s));
    const double t2 = now();
    st->t_setup = t1 - t0;
    st->t_solve = t2 - t1;
    st->t_total = t2 - t0;
    S.finish(st);
    st->status = status;
    if (status != FR_OK) fail_stage(ctx, status);
}

// ---------------------------------------------------------------------------
// full time steps (every stage; the EJ factors formed once at q^n)
// ---------------------------------------------------------------------------

// Tableaux of the full time steps, in pairs of one order that share the
// diagonal gamma (so one shift 1/(gamma dt) and one preconditioner serve both
// schemes of a pair).  The schemes are named in Sec. 2.1 without their
// coefficients; these are derived from the order conditions (Hairer & Wanner,
// Solving ODEs II, Sec. IV.6-IV.7) or taken from their publication.
constexpr int kMaxEsdirkStages = 6, kMaxRowStages = 4;

struct EsdirkTab {
    int s = 0;       // stages, the first explicit; q^{n+1} = q_s (stiffly accurate)
    double g = 0.0;  // a_ii, i >= 1
    double A[kMaxEsdirkStages][kMaxEsdirkStages] = {};
};

struct RowTab {
    int s = 0;
    double g = 0.0;
    // transformed coefficients a = alpha Gamma^{-1}, c = diag(1/gamma) -
    // Gamma^{-1}, m = b Gamma^{-1}
    double a[kMaxRowStages][kMaxRowStages] = {}, c[kMaxRowStages][kMaxRowStages] = {}, m[kMaxRowStages] = {};
};

// order 2: gamma = 1 - 1/sqrt(2) (two implicit stages of order 2 L-stable)
// order 3: gamma = the root in (0.4, 0.5) of 6 g^3 - 18 g^2 + 9 g - 1
// order 4 (ROW): gamma = 1/x, x the second root of the Laguerre polynomial L_4
constexpr double kGamma3 = 0.43586652150845899942;
constexpr double kGamma4 = 0.57281606248213485;

EsdirkTab esdirk_tab(int tableau) {
    EsdirkTab T;
    if (tableau == FR_TAB_ESDIRK2) {
        // c = (0, 2 gamma, 1); b_2 c_2 + gamma = 1/2 and sum b = 1
        // (Kennedy & Carpenter's ESDIRK2(1)3L[2]SA)
        const double g = 1.0 - std::sqrt(0.5);
        const double b2 = (0.5 - g) / (2.0 * g), b1 = 1.0 - b2 - g;
        T.s = 3;
        T.g = g;
        T.A[1][0] = T.A[1][1] = g;
        T.A[2][0] = b1;
        T.A[2][1] = b2;
        T.A[2][2] = g;
    } else if (tableau == FR_TAB_ESDIRK3) {
        // c = (0, 2 gamma, 3/5, 1), the rest fixed by the order-3 conditions
        // (Kennedy & Carpenter's ESDIRK3(2)4L[2]SA)
        const double A[4][4] = {{0.0, 0.0, 0.0, 0.0},
                                {kGamma3, kGamma3, 0.0, 0.0},
                                {0.2576482460664271, -0.09351476757488614, kGamma3, 0.0},
                                {0.18764102434672392, -0.5952974735769553, 0.9717899277217725, kGamma3}};
        T.s = 4;
        T.g = kGamma3;
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) T.A[i][j] = A[i][j];
    } else {
        // six stages, gamma = 1/4: the implicit tableau of Kennedy &
        // Carpenter's ARK4(3)6L[2]SA (the ESDIRK4 of Bijl et al.), published
        // as rationals
        const double g = 0.25;
        const double A[6][6] = {
            {0.0, 0.0, 0.0, 0.0, 0.0, 0.0},
            {g, g, 0.0, 0.0, 0.0, 0.0},
            {8611.0 / 62500.0, -1743.0 / 31250.0, g, 0.0, 0.0, 0.0},
            {5012029.0 / 34652500.0, -654441.0 / 2922500.0, 174375.0 / 388108.0, g, 0.0, 0.0},
            {15267082809.0 / 155376265600.0, -71443401.0 / 120774400.0, 730878875.0 / 902184768.0,
             2285395.0 / 8070912.0, g, 0.0},
            {82889.0 / 524892.0, 0.0, 15625.0 / 83664.0, 69875.0 / 102672.0, -2260.0 / 8211.0, g}};
        T.s = 6;
        T.g = g;
        for (int i = 0; i < 6; ++i)
            for (int j = 0; j < 6; ++j) T.A[i][j] = A[i][j];
    }
    return T;
}

// (alpha, Gamma = beta - alpha + gamma I, b) -> transformed coefficients
RowTab row_transform(int s, double g, const double alpha[kMaxRowStages][kMaxRowStages],
                     const double beta[kMaxRowStages][kMaxRowStages], const double *b) {
    RowTab T;
    T.s = s;
    T.g = g;
    double G[kMaxRowStages][kMaxRowStages] = {}, Gi[kMaxRowStages][kMaxRowStages] = {};
    for (int i = 0; i < s; ++i)
        for (int j = 0; j < i; ++j) G[i][j] = beta[i][j] - alpha[i][j];
    for (int i = 0; i < s; ++i) G[i][i] = g;
    // Gamma^{-1} by forward substitution, column by column
    for (int col = 0; col < s; ++col)
        for (int i = col; i < s; ++i) {
            double t = (i == col) ? 1.0 : 0.0;
            for (int k = col; k < i; ++k) t -= G[i][k] * Gi[k][col];
            Gi[i][col] = t / G[i][i];
        }
    for (int i = 0; i < s; ++i)
        for (int j = 0; j < i; ++j) {
            double t = 0.0;
            for (int k = j; k < i; ++k) t += alpha[i][k] * Gi[k][j];
            T.a[i][j] = t;
            T.c[i][j] = -Gi[i][j];
        }
    for (int j = 0; j < s; ++j) {
        double t = 0.0;
        for (int i = j; i < s; ++i) t += b[i] * Gi[i][j];
        T.m[j] = t;
    }
    return T;
}

RowTab row_tab(int tableau) {
    double al[kMaxRowStages][kMaxRowStages] = {}, be[kMaxRowStages][kMaxRowStages] = {};
    if (tableau == FR_TAB_ROW2) {
        // alpha_21 = 1, b = (1/2, 1/2); sum b beta' = 1/2 - gamma
        const double g = 1.0 - std::sqrt(0.5), b[2] = {0.5, 0.5};
        al[1][0] = 1.0;
        be[1][0] = 1.0 - 2.0 * g;
        return row_transform(2, g, al, be, b);
    }
    if (tableau == FR_TAB_ROW3) {
        // alpha_21 = alpha_31 = 1, alpha_32 = 0, b = (2/3, 1/6, 1/6),
        // beta_31 = beta_21; with s = 3 - 6 gamma, p = 1 - 6 gamma + 6 gamma^2
        // the two remaining order-3 conditions give beta_21 =
        // (s + sqrt(s^2 - 8p))/4, beta_32 = s - 2 beta_21
        const double g = kGamma3, b[3] = {2.0 / 3.0, 1.0 / 6.0, 1.0 / 6.0};
        const double sv = 3.0 - 6.0 * g, pv = 1.0 - 6.0 * g + 6.0 * g * g;
        const double b21 = (sv + std::sqrt(sv * sv - 8.0 * pv)) / 4.0;
        al[1][0] = al[2][0] = 1.0;
        be[1][0] = be[2][0] = b21;
        be[2][1] = sv - 2.0 * b21;
        return row_transform(3, g, al, be, b);
    }
    // ROW4: Shampine's alpha (alpha_21 = 1, alpha_31 = alpha_41 = 12/25,
    // alpha_32 = alpha_42 = 3/25: stages 3 and 4 share one state) and
    // b = (8/27, 1/8, 0, 125/216), gamma_31 = 0, the L-stable gamma of four
    // stages of order 4; the order-4 conditions on beta, taken one at a time
    // (alpha_2 = 1, alpha_3 = alpha_4 = 3/5, b_3 = 0):
    //   b4 alpha_3 alpha_32 beta_21        = 1/8 - g/3
    //   b4 beta_43 beta_32 beta_21         = 1/24 - g/2 + 3g^2/2 - g^3
    //   b4 (beta_42 + alpha_3^2 beta_43)   = 1/12 - g/3
    //   b4 (beta_42 beta_21 + beta_43 beta_3') = 1/6 - g + g^2
    //   b2 beta_21 + b4 beta_4'            = 1/2 - g
    const double g = kGamma4, b[4] = {8.0 / 27.0, 1.0 / 8.0, 0.0, 125.0 / 216.0};
    const double a31 = 12.0 / 25.0, a32 = 3.0 / 25.0, a3 = a31 + a32, b2 = b[1], b4 = b[3];
    const double B21 = (1.0 / 8.0 - g / 3.0) / (b4 * a3 * a32);
    const double prod = (1.0 / 24.0 - g / 2.0 + 1.5 * g * g - g * g * g) / (b4 * B21);  // beta_43 beta_32
    const double S7 = (1.0 / 12.0 - g / 3.0) / b4, Q4 = (1.0 / 6.0 - g + g * g) / b4;
    const double B31 = a31;
    const double B43 = (Q4 - prod - S7 * B21) / (B31 - a3 * a3 * B21);
    const double B32 = prod / B43, B42 = S7 - a3 * a3 * B43;
    const double B41 = (0.5 - g - b2 * B21) / b4 - B42 - B43;
    al[1][0] = 1.0;
    al[2][0] = al[3][0] = a31;
    al[2][1] = al[3][1] = a32;
    be[1][0] = B21;
    be[2][0] = B31;
    be[2][1] = B32;
    be[3][0] = B41;
    be[3][1] = B42;
    be[3][2] = B43;
    return row_transform(4, g, al, be, b);
}

bool is_esdirk_tab(int t) { return t == FR_TAB_ESDIRK2 || t == FR_TAB_ESDIRK3 || t == FR_TAB_ESDIRK4; }
bool is_row_tab(int t) { return t == FR_TAB_ROW2 || t == FR_TAB_ROW3 || t == FR_TAB_ROW4; }

void ensure_step_vectors(frpmg_ctx *ctx, int nvec) {
    const size_t N = ctx->lv[0].N;
    if (ctx->stv && ctx->stv_n >= nvec) return;
    dfree(ctx->stv);
    ctx->stv = dalloc(ctx, (size_t)nvec * N);
    ctx->stv_n = nvec;
    if (!ctx->stw) ctx->stw = dalloc(ctx, N);
}

void step_impl(frpmg_ctx *ctx, const step_params &SP, const double *dq_n, double *out, step_stats *ss,
               hipStream_t s) {
    Range range("time step");
    std::memset(ss, 0, sizeof(*ss));
    const bool esdirk = is_esdirk_tab(SP.tableau);
    REQUIRE(esdirk || is_row_tab(SP.tableau), "unknown tableau");
    REQUIRE(out != dq_n, "the output must not alias q^n");
    const EsdirkTab TE = esdirk ? esdirk_tab(SP.tableau) : EsdirkTab{};
    const RowTab TR = esdirk ? RowTab{} : row_tab(SP.tableau);
    stage_params P = SP.stage;
    P.scheme = esdirk ? FR_SCHEME_ESDIRK : FR_SCHEME_ROW;
    P.a_ii = esdirk ? TE.g : TR.g;
    P.a_i1 = 0.0;
    StageSolver S(ctx, P);
    const size_t N = S.N;
    const int nvec = esdirk ? TE.s - 1 : TR.s;  // ESDIRK: R(q_j), j < s - 1; ROW: Y_i
    ensure_step_vectors(ctx, nvec);
    double *V[kMaxEsdirkStages];
    for (int j = 0; j < nvec; ++j) V[j] = ctx->stv + (size_t)j * N;
    HIPCHK(hipStreamSynchronize(s));
    const double t0 = now();
    S.setup(dq_n, s);
    HIPCHK(hipStreamSynchronize(s));
    const double t1 = now();
    ss->t_setup = t1 - t0;
    fr_status status = FR_OK;
    const Scal one{1.0, nullptr};
    if (esdirk) {
        // stage 1: q_1 = q^n; stages 2..s start from the previous stage's state
        double *q = ctx->sq, *rq = ctx->srq, *b = ctx->sb;
        residual(ctx, 0, dq_n, rq, s);
        S.cnt.R0++;
        HIPCHK(hipMemcpyAsync(V[0], rq, N * sizeof(double), hipMemcpyDeviceToDevice, s));  // R(q_1)
        HIPCHK(hipMemcpyAsync(q, dq_n, N * sizeof(double), hipMemcpyDeviceToDevice, s));
        for (int i = 1; i < TE.s && status == FR_OK; ++i) {
            // b_i = q^n + dt sum_{j<i} a_ij R(q_j)
            HIPCHK(hipMemcpyAsync(b, dq_n, N * sizeof(double), hipMemcpyDeviceToDevice, s));
            for (int j = 0; j < i; ++j)
                if (TE.A[i][j] != 0.0) HIPCHK(vec_axpby(N, Scal{TE.A[i][j] * P.dt, nullptr}, V[j], one, b, s));
            stage_stats *st = &ss->stage[ss->nstages];
            for (double &a : ctx->ph_acc) a = 0.0;
            status = S.esdirk_solve(b, q, rq, st, s);
            st->t_precond = ctx->ph_acc[0];
            st->t_jvp = ctx->ph_acc[1];
            st->t_ortho = ctx->ph_acc[2];
            ss->nstages++;
            ss->gmres_iters += st->gmres_iters;
            ss->ptc_iters += st->ptc_iters;
            if (i < TE.s - 1) HIPCHK(hipMemcpyAsync(V[i], rq, N * sizeof(double), hipMemcpyDeviceToDevice, s));
        }
        HIPCHK(hipMemcpyAsync(out, q, N * sizeof(double), hipMemcpyDeviceToDevice, s));  // stiffly accurate
    } else {
        double *R0 = ctx->srq, *rhs = ctx->sb, *w = ctx->stw, *Rw = ctx->sq;
        residual(ctx, 0, dq_n, R0, s);
        S.cnt.R0++;
        if (S.pmg) {
            pmg_point(ctx, dq_n, R0, s);
            S.cnt.R1 += ctx->nlevels - 1;
        }
        for (int i = 0; i < TR.s && status == FR_OK; ++i) {
            // rhs_i = R(q^n + sum_j a_ij Y_j) + (1/dt) sum_j c_ij Y_j
            if (i == 0) {
                HIPCHK(hipMemcpyAsync(rhs, R0, N * sizeof(double), hipMemcpyDeviceToDevice, s));
            } else {
                bool same = i > 1;
                for (int j = 0; j < TR.s; ++j) same = same && TR.a[i][j] == TR.a[i - 1][j];
                if (!same) {  // stages with the same state share R
                    HIPCHK(hipMemcpyAsync(w, dq_n, N * sizeof(double), hipMemcpyDeviceToDevice, s));
                    for (int j = 0; j < i; ++j)
                        if (TR.a[i][j] != 0.0) HIPCHK(vec_axpby(N, Scal{TR.a[i][j], nullptr}, V[j], one, w, s));
                    residual(ctx, 0, w, Rw, s);
                    S.cnt.R0++;
                }
                HIPCHK(hipMemcpyAsync(rhs, Rw, N * sizeof(double), hipMemcpyDeviceToDevice, s));
                for (int j = 0; j < i; ++j)
                    if (TR.c[i][j] != 0.0) HIPCHK(vec_axpby(N, Scal{TR.c[i][j] / P.dt, nullptr}, V[j], one, rhs, s));
            }
            stage_stats *st = &ss->stage[ss->nstages];
            for (double &a : ctx->ph_acc) a = 0.0;
            status = S.row_solve(dq_n, R0, rhs, V[i], st, s);
            st->t_precond = ctx->ph_acc[0];
            st->t_jvp = ctx->ph_acc[1];
            st->t_ortho = ctx->ph_acc[2];
            ss->nstages++;
            ss->gmres_iters += st->gmres_iters;
        }
        HIPCHK(hipMemcpyAsync(out, dq_n, N * sizeof(double), hipMemcpyDeviceToDevice, s));
        for (int i = 0; i < TR.s; ++i) HIPCHK(vec_axpby(N, Scal{TR.m[i], nullptr}, V[i], one, out, s));
    }
    HIPCHK(hipStreamSynchronize(s));
    const double t2 = now();
    ss->t_solve = t2 - t1;
    ss->t_total = t2 - t0;
    ss->n_R_fine = S.cnt.R0;
    ss->n_R_coarse = S.cnt.R1;
    ss->n_ej_fine = S.cnt.E0;
    ss->n_ej_coarse = S.cnt.E1;
    ss->fallbacks = S.fallbacks;
    ss->status = status;
    if (status != FR_OK) fail_stage(ctx, status);
}

// ---------------------------------------------------------------------------
// mixed polynomial degrees (p-adaptation, Sec. 3.3)
// ---------------------------------------------------------------------------

void pa_free_level(Level &L) {
    if (!L.pa) return;
    PaLevel &pa = *L.pa;
    dfree(pa.Pk);
    dfree(pa.cls);
    dfree(pa.mixed);
    dfree(pa.Fm);
    dfree(pa.Mq);
    dfree(pa.Mn);
    dfree(pa.Mg);
    dfree(pa.PkB);
    dfree(pa.clsB);
    dfree(pa.mixedB);
    double *bb[] = {pa.JpB, pa.FsB, pa.FmB, pa.MqB, pa.MnB, pa.MgB, pa.qB, pa.rB};
    for (double *b : bb) dfree(b);
    delete L.pa;
    L.pa = nullptr;
}

// Degrees of every element on each p-sublevel of a nested hierarchy (order
// gap 1 or 2): each sublevel lowers the finest degree by the gap, keeps at
// least as many degrees as sublevels remain below it, stays below the
// sublevel above and stops at 0 (Sec. 3.3 lists the hierarchies this gives
// for P4 down to P1 with three sublevels).
void pa_nested(const int *deg, int ne, int nlev, int gap, int *out) {
    for (int k = 0; k < ne; ++k) {
        int prev = deg[k];
        out[k] = prev;
        for (int l = 1; l < nlev; ++l) {
            int pl = std::min(prev - 1, std::max(deg[k] - gap * l, nlev - 1 - l));
            pl = std::max(pl, 0);
            out[(size_t)l * ne + k] = pl;
            prev = pl;
        }
    }
}

void ensure_pa_tables(frpmg_ctx *ctx) {
    if (ctx->pa_tab) return;
    ctx->pa_tab_host = new PaTables();
    build_pa_tables(*ctx->pa_tab_host);
    void *p = nullptr;
    HIPCHK(hipMalloc(&p, sizeof(PaTables)));
    ctx->pa_tab = (PaTables *)p;
    HIPCHK(hipMemcpy(ctx->pa_tab, ctx->pa_tab_host, sizeof(PaTables), hipMemcpyHostToDevice));
}

void pa_build_level(frpmg_ctx *ctx, int l, const int *deg) {
    Level &L = ctx->lv[l];
    const MeshK &m = ctx->mesh;
    const int Ne = m.Ne;
    pa_free_level(L);
    L.pa = new PaLevel();
    PaLevel &pa = *L.pa;
    pa.Pk_host.resize(Ne);
    std::vector<int> cls;
    cls.reserve(Ne);
    for (int P = 1; P <= kMaxP; ++P) {
        pa.cls_off[P] = (int)cls.size();
        for (int k = 0; k < Ne; ++k)
            if (deg[k] + 1 == P) cls.push_back(k);
    }
    pa.cls_off[kMaxP + 1] = (int)cls.size();
    std::vector<int> mixed;
    for (int k = 0; k < Ne; ++k) {
        pa.Pk_host[k] = deg[k] + 1;
        int c[3] = {k % m.n[0], (k / m.n[0]) % m.n[1], (ctx->dim == 3) ? k / (m.n[0] * m.n[1]) : 0};
        for (int a = 0; a < ctx->dim; ++a) {
            int d[3] = {c[0], c[1], c[2]};
            d[a] = (d[a] + 1) % m.n[a];
            const int kn = d[0] + m.n[0] * (d[1] + m.n[1] * d[2]);
            if (deg[kn] != deg[k]) mixed.push_back(k * 4 + a);
        }
    }
    pa.nmixed = (int)mixed.size();
    void *p = nullptr;
    HIPCHK(hipMalloc(&p, (size_t)Ne * sizeof(int)));
    pa.Pk = (int *)p;
    HIPCHK(hipMemcpy(pa.Pk, pa.Pk_host.data(), (size_t)Ne * sizeof(int), hipMemcpyHostToDevice));
    HIPCHK(hipMalloc(&p, (size_t)Ne * sizeof(int)));
    pa.cls = (int *)p;
    HIPCHK(hipMemcpy(pa.cls, cls.data(), (size_t)Ne * sizeof(int), hipMemcpyHostToDevice));
    if (pa.nmixed > 0) {
        HIPCHK(hipMalloc(&p, (size_t)pa.nmixed * sizeof(int)));
        pa.mixed = (int *)p;
        HIPCHK(hipMemcpy(pa.mixed, mixed.data(), (size_t)pa.nmixed * sizeof(int), hipMemcpyHostToDevice));
    }
    const size_t nface = (size_t)ctx->dim * ctx->nv * L.NF * Ne;
    pa.Fm = dalloc(ctx, nface);
    pa.Mq = dalloc(ctx, nface);
    pa.Mn = dalloc(ctx, nface);
    pa.Mg = dalloc(ctx, nface * ctx->dim);
    // copies for the coloured-difference EJ formation: as many (colour,
    // column) perturbations per evaluation as fit in 512 MiB, at most 64
    const size_t per_copy = (2 * L.N + (5 + (size_t)ctx->dim) * nface) * sizeof(double) + 2 * (size_t)Ne * sizeof(int);
    const long npairs = (long)(1 << ctx->dim) * L.nb;
    long B = (long)((size_t(512) << 20) / per_copy);
    B = std::max(1L, std::min({B, 64L, npairs}));
    if ((long)Ne * B >= (1L << 29)) B = std::max(1L, ((1L << 29) - 1) / Ne);  // face codes (id * 4 + axis) stay in an int
    pa.fdB = (int)B;
    std::vector<int> PkB((size_t)B * Ne), clsB;
    std::vector<int> mixedB;
    clsB.reserve((size_t)B * Ne);
    for (long b = 0; b < B; ++b)
        for (int k = 0; k < Ne; ++k) PkB[(size_t)b * Ne + k] = pa.Pk_host[k];
    for (int P = 1; P <= kMaxP; ++P) {
        pa.clsB_off[P] = (int)clsB.size();
        for (long b = 0; b < B; ++b)
            for (int u = pa.cls_off[P]; u < pa.cls_off[P + 1]; ++u) clsB.push_back((int)(b * Ne) + cls[u]);
    }
    pa.clsB_off[kMaxP + 1] = (int)clsB.size();
    for (long b = 0; b < B; ++b)
        for (int code : mixed) mixedB.push_back(((int)(b * Ne) + (code >> 2)) * 4 + (code & 3));
    HIPCHK(hipMalloc(&p, PkB.size() * sizeof(int)));
    pa.PkB = (int *)p;
    HIPCHK(hipMemcpy(pa.PkB, PkB.data(), PkB.size() * sizeof(int), hipMemcpyHostToDevice));
    HIPCHK(hipMalloc(&p, clsB.size() * sizeof(int)));
    pa.clsB = (int *)p;
    HIPCHK(hipMemcpy(pa.clsB, clsB.data(), clsB.size() * sizeof(int), hipMemcpyHostToDevice));
    if (!mixedB.empty()) {
        HIPCHK(hipMalloc(&p, mixedB.size() * sizeof(int)));
        pa.mixedB = (int *)p;
        HIPCHK(hipMemcpy(pa.mixedB, mixedB.data(), mixedB.size() * sizeof(int), hipMemcpyHostToDevice));
    }
    pa.JpB = dalloc(ctx, nface * B);
    pa.FsB = dalloc(ctx, nface * B);
    pa.FmB = dalloc(ctx, nface * B);
    pa.MqB = dalloc(ctx, nface * B);
    pa.MnB = dalloc(ctx, nface * B);
    pa.MgB = dalloc(ctx, nface * ctx->dim * B);
    pa.qB = dalloc(ctx, L.N * B);
    pa.rB = dalloc(ctx, L.N * B);
}

void destroy_all(frpmg_ctx *ctx) {
    clear_graphs(ctx);
    for (auto &e : ctx->ph_ev) {
        if (e) (void)hipEventDestroy(e);
        e = nullptr;
    }
    for (auto &e : ctx->step_ev) {
        if (e) (void)hipEventDestroy(e);
        e = nullptr;
    }
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    ctx->cap_stream = nullptr;
    lcc_free(ctx);
    mbnk_free(ctx);
    for (int l = 0; l < FR_MAX_LEVELS; ++l) pa_free_level(ctx->lv[l]);
    dfree(ctx->pa_tab);
    delete ctx->pa_tab_host;
    ctx->pa_tab_host = nullptr;
    for (int l = 0; l < FR_MAX_LEVELS; ++l) {
        Level &L = ctx->lv[l];
        dfree(L.Jp);
        dfree(L.Fs);
        dfree(L.fQs);
        dfree(L.fQp);
        dfree(L.fSn);
        dfree(L.fGt);
        dfree(L.blk64);
        dfree(L.inv32);
        dfree(L.inv16);
        dfree(L.dstatus);
        dfree(L.perm);
        dfree(L.touch);
        dfree(L.colperm);
        dfree(L.r0);
    }
    for (int l = 2; l < FR_MAX_LEVELS; ++l) {  // level 1 is freed through its names below
        double *lb[] = {ctx->mq[l], ctx->mr[l], ctx->mZ0[l], ctx->mZ[l], ctx->mS[l], ctx->mG[l], ctx->md[l]};
        for (double *b : lb) dfree(b);
    }
    for (int a = 0; a < 3; ++a) dfree(ctx->inv2h[a]);
    dfree(ctx->red_partial);
    dfree(ctx->red_out);
    dfree(ctx->scal);
    if (ctx->host_pinned) (void)hipHostFree(ctx->host_pinned);
    if (ctx->host_pinned2) (void)hipHostFree(ctx->host_pinned2);
    double *bufs[] = {ctx->q1, ctx->r1, ctx->wY, ctx->wG, ctx->wXs, ctx->cZ0, ctx->cZ, ctx->cS, ctx->cG, ctx->cd,
                      ctx->V, ctx->Zk, ctx->kw, ctx->sq, ctx->srq, ctx->sF, ctx->sb, ctx->sdx,
                      ctx->stv, ctx->stw};
    for (double *b : bufs) dfree(b);
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================

extern "C" {

fr_status fr_create(const fr_mesh_desc *d, frpmg_ctx **out) {
    if (!d || !out) return FR_EINVAL;
    *out = nullptr;
    frpmg_ctx *ctx = new (std::nothrow) frpmg_ctx();
    if (!ctx) return FR_ENOMEM;
    fr_status st = guarded(ctx, [&] {
        REQUIRE(d->dim == 2 || d->dim == 3, "dim must be 2 or 3");
        REQUIRE(d->nlevels >= 1 && d->nlevels <= FR_MAX_LEVELS, "nlevels out of range");
        ctx->dim = d->dim;
        ctx->nv = d->dim + 2;
        ctx->nlevels = d->nlevels;
        MeshK &m = ctx->mesh;
        m.dim = d->dim;
        m.n[2] = 1;
        long ne = 1;
        for (int a = 0; a < d->dim; ++a) {
            REQUIRE(d->n[a] >= 1, "element counts must be >= 1");
            REQUIRE(d->h[a] != nullptr, "element widths missing");
            m.n[a] = d->n[a];
            ne *= d->n[a];
        }
        REQUIRE(ne < (1L << 30), "too many elements");
        m.Ne = (int)ne;
        for (int a = 0; a < 3; ++a) {
            REQUIRE((unsigned long long)ne * (unsigned long long)m.n[a] < (1ULL << 40), "mesh too large");
            m.rcp[a] = ((1ULL << 40) + (unsigned long long)m.n[a] - 1) / (unsigned long long)m.n[a];
        }
        for (int a = 0; a < d->dim; ++a) {
            std::vector<double> ih(d->n[a]);
            for (int i = 0; i < d->n[a]; ++i) {
                REQUIRE(d->h[a][i] > 0.0, "element widths must be positive");
                ih[i] = 2.0 / d->h[a][i];
            }
            ctx->inv2h[a] = dalloc(ctx, d->n[a]);
            HIPCHK(hipMemcpy(ctx->inv2h[a], ih.data(), d->n[a] * sizeof(double), hipMemcpyHostToDevice));
            m.inv2h[a] = ctx->inv2h[a];
        }
        for (int a = d->dim; a < 3; ++a) m.inv2h[a] = nullptr;
        Phys &ph = ctx->phys;
        ph.gam = d->gamma;
        ph.mu = d->mu;
        ph.Pr = d->Pr;
        ph.tau = d->tau;
        REQUIRE(d->qinf[0] > 0.0, "reference density must be positive");
        double kin = 0.0;
        for (int v = 0; v < 5; ++v) ph.qinf[v] = (v < ctx->nv) ? d->qinf[v] : 0.0;
        for (int b = 0; b < 3; ++b) ph.uinf[b] = (b < d->dim) ? d->qinf[1 + b] / d->qinf[0] : 0.0;
        for (int b = 0; b < d->dim; ++b) kin += d->qinf[1 + b] * ph.uinf[b];
        ph.pinf = (d->gamma - 1.0) * (d->qinf[d->dim + 1] - 0.5 * kin);
        REQUIRE(ph.pinf > 0.0, "reference pressure must be positive");
        for (int l = 0; l < d->nlevels; ++l) {
            const int p = d->p[l];
            REQUIRE(p >= 0 && p <= (d->dim == 2 ? 4 : 3), "polynomial degree out of range");
            if (l > 0) REQUIRE(p < d->p[l - 1], "levels must have decreasing degree");
            Level &L = ctx->lv[l];
            L.p = p;
            L.P = p + 1;
            L.Np = ipow(L.P, d->dim);
            L.NF = ipow(L.P, d->dim - 1);
            L.nb = ctx->nv * L.Np;
            L.N = (size_t)L.nb * m.Ne;
            build_ops1d(L.P, L.ops);
            const size_t ntr = (size_t)d->dim * ctx->nv * L.NF * m.Ne;
            L.Jp = dalloc(ctx, ntr);
            L.Fs = dalloc(ctx, ntr);
            L.r0 = dalloc(ctx, L.N);
            void *p2 = nullptr;
            HIPCHK(hipMalloc(&p2, sizeof(int)));
            L.dstatus = (int *)p2;
            if (l > 0) build_transfer(ctx->lv[l - 1].P, L.P, ctx->tr[l - 1]);
        }
        ctx->red_partial = dalloc(ctx, (size_t)128 * kRedBlocks);
        ctx->red_out = dalloc(ctx, RO_SIZE);
        ctx->scal = dalloc(ctx, 16);
        void *hp = nullptr;
        HIPCHK(hipHostMalloc(&hp, RO_SIZE * sizeof(double), hipHostMallocDefault));
        ctx->host_pinned = (double *)hp;
        HIPCHK(hipHostMalloc(&hp, RO_SIZE * sizeof(double), hipHostMallocDefault));
        ctx->host_pinned2 = (double *)hp;
        const size_t N0 = ctx->lv[0].N;
        ctx->wY = dalloc(ctx, N0);
        ctx->wG = dalloc(ctx, N0);
        ctx->wXs = dalloc(ctx, N0);
        for (int l = 1; l < d->nlevels; ++l) {
            const size_t Nl = ctx->lv[l].N;
            ctx->mq[l] = dalloc(ctx, Nl);
            ctx->mr[l] = dalloc(ctx, Nl);
            ctx->mZ0[l] = dalloc(ctx, Nl);
            ctx->mZ[l] = dalloc(ctx, Nl);
            ctx->mS[l] = dalloc(ctx, Nl);
            ctx->mG[l] = dalloc(ctx, Nl);
            ctx->md[l] = dalloc(ctx, Nl);
        }
        {
            int dev = 0;
            HIPCHK(hipGetDevice(&dev));
            REQUIRE(dev >= 0 && dev < kMaxDevices, "device index out of range");
            std::lock_guard<std::mutex> lock(g_scratch_mu);
            if (!g_scratch_addr[dev]) {
                double *ptr = nullptr;
                HIPCHK(hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch)));
                g_scratch_addr[dev] = ptr;
            }
            ctx->noalloc_scratch = g_scratch_addr[dev];
        }
        if (d->nlevels > 1) {
            ctx->q1 = ctx->mq[1];
            ctx->r1 = ctx->mr[1];
            ctx->cZ0 = ctx->mZ0[1];
            ctx->cZ = ctx->mZ[1];
            ctx->cS = ctx->mS[1];
            ctx->cG = ctx->mG[1];
            ctx->cd = ctx->md[1];
        }
        HIPCHK(hipDeviceSynchronize());
    });
    if (st != FR_OK) {
        std::fprintf(stderr, "fr_create: %s\n", ctx->err.c_str());
        destroy_all(ctx);
        delete ctx;
        return st;
    }
    *out = ctx;
    return FR_OK;
}

void fr_destroy(frpmg_ctx *ctx) {
    if (!ctx) return;
    (void)hipDeviceSynchronize();
    destroy_all(ctx);
    delete ctx;
}

const char *fr_last_error(const frpmg_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

size_t fr_level_size(const frpmg_ctx *ctx, int level) {
    if (!ctx || level < 0 || level >= ctx->nlevels) return 0;
    return ctx->lv[level].N;
}

fr_status fr_residual(frpmg_ctx *ctx, int level, const double *dq, double *r, fr_stream stream) {
    return guarded(ctx, [&] {
        REQUIRE(level >= 0 && level < ctx->nlevels, "bad level");
        REQUIRE(dq && r && dq != r, "bad pointers");
        residual(ctx, level, dq, r, S(stream));
    });
}

fr_status fr_residual_noalloc(frpmg_ctx *ctx, int level, const double *dq, double *r, fr_stream stream) {
    return guarded(ctx, [&] {
        REQUIRE(level >= 0 && level < ctx->nlevels, "bad level");
        REQUIRE(dq && r && dq != r, "bad pointers");
        REQUIRE(ctx->noalloc_scratch, "no scratch address for this device");
        const Level &L = ctx->lv[level];
        REQUIRE(!L.pa, "fr_residual_noalloc takes uniform-degree levels");
        // common fluxes, then state jumps, each [dim][nv][NF][Ne], the second 256-byte aligned
        const size_t nface = ((size_t)ctx->dim * ctx->nv * L.NF * ctx->mesh.Ne + 31) / 32 * 32;
        if (2 * nface * sizeof(double) > kNoallocBytes) {
            char msg[160];
            std::snprintf(msg, sizeof msg, "fr_residual_noalloc: the level's face data (%zu bytes) exceed the %zu-byte "
                          "scratch", 2 * nface * sizeof(double), kNoallocBytes);
            ctx->err = msg;
            throw Fail{FR_EINVAL};
        }
        double *Fs = ctx->noalloc_scratch, *Jp = ctx->noalloc_scratch + nface;
        HIPCHK(launch_residual_batch(ctx, level, 1, dq, r, Jp, Fs, S(stream)));
    });
}

fr_status fr_jvp(frpmg_ctx *ctx, int level, const double *dq, const double *rq, const double *v, double shift,
                 double eps, int eps_mode, double *w, fr_stream stream) {
    return guarded(ctx, [&] {
        REQUIRE(level >= 0 && level < ctx->nlevels, "bad level");
        REQUIRE(dq && rq && v && w, "null pointer");
        REQUIRE(w != dq && w != rq && w != v, "w must not alias the inputs");
        REQUIRE(eps > 0.0, "eps must be positive");
        REQUIRE(valid_eps_mode(eps_mode), "bad eps_mode");
        jvp(ctx, level, dq, rq, v, shift, eps, eps_mode, w, S(stream));
    });
}

fr_status ej_factor(frpmg_ctx *ctx, int level, const double *dq_lin, double sigma, int precision,
                    fr_stream stream) {
    return guarded(ctx, [&] {
        REQUIRE(dq_lin, "null pointer");
        ej_factor_impl(ctx, level, dq_lin, sigma, precision, S(stream));
    });
}

fr_status ej_solve(frpmg_ctx *ctx, int level, const double *r, double *y, fr_stream stream) {
    return guarded(ctx, [&] {
        REQUIRE(level >= 0 && level < ctx->nlevels, "bad level");
        REQUIRE(ctx->lv[level].inv_prec >= 0, "level has no EJ factors");
        REQUIRE(r && y, "null pointer");
        HIPCHK(ej_apply(ctx, level, r, 1.0, 0.0, y, S(stream)));
    });
}

fr_status ej_get_inverse(frpmg_ctx *ctx, int level, double *host_out) {
    return guarded(ctx, [&] {
        REQUIRE(level >= 0 && level < ctx->nlevels, "bad level");
        const Level &L = ctx->lv[level];
        REQUIRE(L.inv_prec >= 0, "level has no EJ factors");
        REQUIRE(host_out, "null pointer");
        const size_t n = (size_t)ctx->mesh.Ne * L.nb * L.nb;
        HIPCHK(hipDeviceSynchronize());
        if (L.inv_prec == FR_PREC_FP64) {
            HIPCHK(hipMemcpy(host_out, L.inv, n * sizeof(double), hipMemcpyDeviceToHost));
        } else if (L.inv_prec == FR_PREC_BF16_STORE) {
            std::vector<uint16_t> tmp(n);
            HIPCHK(hipMemcpy(tmp.data(), L.inv, n * sizeof(uint16_t), hipMemcpyDeviceToHost));
            for (size_t i = 0; i < n; ++i) {
                const uint32_t bits = (uint32_t)tmp[i] << 16;
                float f;
                std::memcpy(&f, &bits, sizeof(f));
                host_out[i] = f;
            }
        } else {
            std::vector<float> tmp(n);
            HIPCHK(hipMemcpy(tmp.data(), L.inv, n * sizeof(float), hipMemcpyDeviceToHost));
            for (size_t i = 0; i < n; ++i) host_out[i] = tmp[i];
        }
        if (L.inv_cols) {
            // stored column j is column inv_cols[j] of the inverse
            const int nb = L.nb;
            std::vector<int> cols((size_t)ctx->mesh.Ne * nb);
            HIPCHK(hipMemcpy(cols.data(), L.inv_cols, cols.size() * sizeof(int), hipMemcpyDeviceToHost));
            std::vector<double> blk((size_t)nb * nb);
            for (int k = 0; k < ctx->mesh.Ne; ++k) {
                double *Bk = host_out + (size_t)k * nb * nb;
                std::memcpy(blk.data(), Bk, blk.size() * sizeof(double));
                for (int j = 0; j < nb; ++j)
                    std::memcpy(Bk + (size_t)cols[(size_t)k * nb + j] * nb, blk.data() + (size_t)j * nb,
                                nb * sizeof(double));
            }
        }
    });
}

fr_status mbnk_factor(frpmg_ctx *ctx, int level, const double *dq_lin, double sigma, fr_stream stream) {
    return guarded(ctx, [&] {
        REQUIRE(dq_lin, "null pointer");
        mbnk_factor_impl(ctx, level, dq_lin, sigma, S(stream));
    });
}

fr_status mbnk_matvec(frpmg_ctx *ctx, const double *x, double *y, fr_stream stream) {
    return guarded(ctx, [&] {
        REQUIRE(x && y && x != y, "bad pointers");
        HIPCHK(mb_matvec(ctx, mbnk_of(ctx, -1), x, y, S(stream)));
    });
}

fr_status mbnk_ilu_solve(frpmg_ctx *ctx, const double *r, double *z, fr_stream stream) {
    return guarded(ctx, [&] {
        REQUIRE(r && z && r != z, "bad pointers");
        HIPCHK(mb_ilu(ctx, mbnk_of(ctx, -1), r, z, S(stream)));
    });
}

fr_status mbnk_solve(frpmg_ctx *ctx, const double *g, double *delta, double tol, int maxit, fr_stream stream) {
    return guarded(ctx, [&] {
        REQUIRE(g && delta, "null pointer");
        REQUIRE(maxit >= 1 && maxit <= kMbnkMaxIt, "maxit must be in 1..8");
        REQUIRE(tol >= 0.0, "tol must be non-negative");
        HIPCHK(mb_sweep(ctx, mbnk_of(ctx, -1), g, nullptr, delta, tol, maxit, S(stream)));
    });
}

fr_status mbnk_get_blocks(frpmg_ctx *ctx, double *host_D, double *host_O) {
    return guarded(ctx, [&] {
        const Mbnk &mb = mbnk_of(ctx, -1);
        const size_t nn = (size_t)mb.nb * mb.nb;
        HIPCHK(hipDeviceSynchronize());
        if (host_D) HIPCHK(hipMemcpy(host_D, mb.D, (size_t)mb.Ne * nn * sizeof(double), hipMemcpyDeviceToHost));
        if (host_O)
            HIPCHK(hipMemcpy(host_O, mb.O, (size_t)mb.Ne * mb.nface * nn * sizeof(double), hipMemcpyDeviceToHost));
    });
}

fr_status pmg_restrict(frpmg_ctx *ctx, int from, int to, const double *x, double *y, fr_stream stream) {
    return guarded(ctx, [&] {
        REQUIRE(from >= 0 && to == from + 1 && to < ctx->nlevels, "restriction goes from level l to l + 1");
        REQUIRE(x && y && x != y, "bad pointers");
        HIPCHK(transfer_apply(ctx, from, true, x, y, S(stream)));
    });
}

fr_status pmg_prolong(frpmg_ctx *ctx, int from, int to, const double *x, double *y, fr_stream stream) {
    return guarded(ctx, [&] {
        REQUIRE(to >= 0 && from == to + 1 && from < ctx->nlevels, "prolongation goes from level l + 1 to l");
        REQUIRE(x && y && x != y, "bad pointers");
        HIPCHK(transfer_apply(ctx, to, false, x, y, S(stream)));
    });
}

fr_status pmg_set_point(frpmg_ctx *ctx, const double *dq, const double *rq, fr_stream stream) {
    return guarded(ctx, [&] {
        REQUIRE(dq && rq, "null pointer");
        pmg_point(ctx, dq, rq, S(stream));
    });
}

fr_status pmg_precond_apply(frpmg_ctx *ctx, const pmg_params *prm, const double *x, double *y, fr_stream stream) {
    return guarded(ctx, [&] {
        REQUIRE(prm && x && y && x != y, "bad arguments");
        Counters c;
        pmg_apply_impl(ctx, *prm, x, y, S(stream), &c);
    });
}

fr_status gmres_solve_stage(frpmg_ctx *ctx, const stage_params *prm, const double *dq_n, double *out,
                            stage_stats *stats, fr_stream stream) {
    stage_stats local;
    stage_stats *st = stats ? stats : &local;
    return guarded(ctx, [&] {
        REQUIRE(prm && dq_n && out && dq_n != out, "bad arguments");
        stage_impl(ctx, *prm, dq_n, out, st, S(stream));
    });
}

fr_status fr_time_step(frpmg_ctx *ctx, const step_params *prm, const double *dq_n, double *dq_np1,
                       step_stats *stats, fr_stream stream) {
    step_stats local;
    step_stats *st = stats ? stats : &local;
    return guarded(ctx, [&] {
        REQUIRE(prm && dq_n && dq_np1 && dq_n != dq_np1, "bad arguments");
        step_impl(ctx, *prm, dq_n, dq_np1, st, S(stream));
    });
}

fr_status fr_step_tableau(int tableau, fr_tableau *out) {
    if (!out || !(is_esdirk_tab(tableau) || is_row_tab(tableau))) return FR_EINVAL;
    std::memset(out, 0, sizeof(*out));
    if (is_esdirk_tab(tableau)) {
        const EsdirkTab T = esdirk_tab(tableau);
        out->stages = T.s;
        out->gamma = T.g;
        for (int i = 0; i < T.s; ++i)
            for (int j = 0; j < T.s; ++j) out->A[i][j] = T.A[i][j];
    } else {
        const RowTab T = row_tab(tableau);
        out->rosenbrock = 1;
        out->stages = T.s;
        out->gamma = T.g;
        for (int i = 0; i < T.s; ++i) {
            for (int j = 0; j < T.s; ++j) {
                out->a[i][j] = T.a[i][j];
                out->c[i][j] = T.c[i][j];
            }
            out->m[i] = T.m[i];
        }
    }
    return FR_OK;
}

fr_status lcc_harvest(frpmg_ctx *ctx, const lcc_harvest_params *prm) {
    return guarded(ctx, [&] {
        REQUIRE(prm, "null parameters");
        lcc_alloc(ctx);
        Lcc &L = *ctx->lcc;
        if (prm->reset) {
            L.count = 0;
            L.cycle = 0;
            L.scales_set = 0;
        }
        if (prm->enable) {
            REQUIRE(prm->max_pairs > 0 && prm->stride >= 1 && prm->target_sweeps >= 1, "bad harvest parameters");
            if (!L.HX || prm->max_pairs != L.cap) {
                // new capacity: the pairs harvested so far (up to the new capacity) move over
                float *hx = talloc<float>(ctx, (size_t)prm->max_pairs * L.nin_pad);
                float *ht = talloc<float>(ctx, (size_t)prm->max_pairs * L.nout_pad);
                const int keep = L.HX ? std::min(L.count, prm->max_pairs) : 0;
                HIPCHK(hipDeviceSynchronize());
                if (keep > 0) {
                    HIPCHK(hipMemcpy(hx, L.HX, (size_t)keep * L.nin_pad * sizeof(float), hipMemcpyDeviceToDevice));
                    HIPCHK(hipMemcpy(ht, L.HT, (size_t)keep * L.nout_pad * sizeof(float), hipMemcpyDeviceToDevice));
                }
                dfree(L.HX);
                dfree(L.HT);
                L.HX = hx;
                L.HT = ht;
                L.cap = prm->max_pairs;
                L.count = keep;
            }
            L.stride = prm->stride;
            L.target_sweeps = prm->target_sweeps;
        }
        L.harvesting = prm->enable ? 1 : 0;
    });
}

int lcc_harvest_count(const frpmg_ctx *ctx) { return (ctx && ctx->lcc) ? ctx->lcc->count : 0; }

fr_status lcc_dims(frpmg_ctx *ctx, int *nin, int *nin_pad, int *nh, int *nout, int *nout_pad) {
    return guarded(ctx, [&] {
        lcc_alloc(ctx);
        const Lcc &L = *ctx->lcc;
        if (nin) *nin = L.nin;
        if (nin_pad) *nin_pad = L.nin_pad;
        if (nh) *nh = L.nh;
        if (nout) *nout = L.nout;
        if (nout_pad) *nout_pad = L.nout_pad;
    });
}

size_t lcc_num_weights(frpmg_ctx *ctx) {
    if (!ctx || lcc_dims(ctx, nullptr, nullptr, nullptr, nullptr, nullptr) != FR_OK) return 0;
    const Lcc &L = *ctx->lcc;
    size_t n = 0;
    for (int l = 0; l < 3; ++l) n += (size_t)L.wrows[l] * L.wcols[l];
    return n;
}

fr_status lcc_get_weights(frpmg_ctx *ctx, float *host, size_t n) {
    return guarded(ctx, [&] {
        REQUIRE(host && n == lcc_num_weights(ctx), "weight buffer size mismatch");
        Lcc &L = *ctx->lcc;
        HIPCHK(hipDeviceSynchronize());
        size_t off = 0;
        for (int l = 0; l < 3; ++l) {
            const size_t m = (size_t)L.wrows[l] * L.wcols[l];
            HIPCHK(hipMemcpy(host + off, L.W[l], m * sizeof(float), hipMemcpyDeviceToHost));
            off += m;
        }
    });
}

fr_status lcc_set_weights(frpmg_ctx *ctx, const float *host, size_t n) {
    return guarded(ctx, [&] {
        REQUIRE(host && n == lcc_num_weights(ctx), "weight buffer size mismatch");
        Lcc &L = *ctx->lcc;
        HIPCHK(hipDeviceSynchronize());
        size_t off = 0;
        for (int l = 0; l < 3; ++l) {
            const size_t m = (size_t)L.wrows[l] * L.wcols[l];
            HIPCHK(hipMemcpy(L.W[l], host + off, m * sizeof(float), hipMemcpyHostToDevice));
            HIPCHK(hipMemset(L.Mo[l], 0, m * sizeof(float)));
            HIPCHK(hipMemset(L.Vo[l], 0, m * sizeof(float)));
            HIPCHK(lcc_to_bf(m, L.W[l], L.Wb[l], nullptr));
            off += m;
        }
        L.adam_step = 0;
        HIPCHK(hipDeviceSynchronize());
    });
}

fr_status lcc_get_scales(frpmg_ctx *ctx, float *in_scale, float *out_scale) {
    return guarded(ctx, [&] {
        lcc_alloc(ctx);
        REQUIRE(ctx->lcc->scales_set, "scales not set");
        for (int v = 0; v < ctx->nv; ++v) {
            if (in_scale) in_scale[v] = ctx->lcc->h_in_scale[v];
            if (out_scale) out_scale[v] = ctx->lcc->h_out_scale[v];
        }
    });
}

fr_status lcc_set_scales(frpmg_ctx *ctx, const float *in_scale, const float *out_scale) {
    return guarded(ctx, [&] {
        REQUIRE(in_scale && out_scale, "null scales");
        lcc_alloc(ctx);
        Lcc &L = *ctx->lcc;
        for (int v = 0; v < ctx->nv; ++v) {
            REQUIRE(in_scale[v] > 0.f && out_scale[v] > 0.f, "scales must be positive");
            L.h_in_scale[v] = in_scale[v];
            L.h_out_scale[v] = out_scale[v];
        }
        HIPCHK(hipMemcpy(L.in_scale, L.h_in_scale, 5 * sizeof(float), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(L.out_scale, L.h_out_scale, 5 * sizeof(float), hipMemcpyHostToDevice));
        L.scales_set = 1;
    });
}

fr_status lcc_forward(frpmg_ctx *ctx, const float *X, int rows, float *Y, fr_stream stream) {
    return guarded(ctx, [&] {
        REQUIRE(X && Y && rows > 0 && rows % 32 == 0, "rows must be a positive multiple of 32");
        lcc_alloc(ctx);
        lcc_train_buffers(ctx, rows);
        Lcc &L = *ctx->lcc;
        hipStream_t s = S(stream);
        HIPCHK(lcc_to_bf((size_t)rows * L.nin_pad, X, L.bX, s));
        lcc_forward_rows(ctx, rows, L.bX, L.bH1, L.bH2, L.bY, s);
        HIPCHK(hipMemcpyAsync(Y, L.bY, (size_t)rows * L.nout_pad * sizeof(float), hipMemcpyDeviceToDevice, s));
    });
}

fr_status lcc_loss_grad(frpmg_ctx *ctx, const float *X, const float *T, int rows, double *loss, float *grad,
                        fr_stream stream) {
    return guarded(ctx, [&] {
        REQUIRE(X && T && grad && loss && rows > 0 && rows % 32 == 0, "bad arguments");
        lcc_alloc(ctx);
        lcc_train_buffers(ctx, rows);
        Lcc &L = *ctx->lcc;
        hipStream_t s = S(stream);
        HIPCHK(lcc_to_bf((size_t)rows * L.nin_pad, X, L.bX, s));
        HIPCHK(hipMemcpyAsync(L.bT, T, (size_t)rows * L.nout_pad * sizeof(float), hipMemcpyDeviceToDevice, s));
        lcc_batch_grad(ctx, s);
        size_t off = 0;
        for (int l = 0; l < 3; ++l) {
            const size_t m = (size_t)L.wrows[l] * L.wcols[l];
            HIPCHK(hipMemcpyAsync(grad + off, L.G[l], m * sizeof(float), hipMemcpyDeviceToDevice, s));
            off += m;
        }
        HIPCHK(hipMemcpyAsync(ctx->host_pinned, L.lval, sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        *loss = ctx->host_pinned[0];
    });
}

fr_status lcc_adam_step(frpmg_ctx *ctx, const float *grad, double lr, fr_stream stream) {
    return guarded(ctx, [&] {
        REQUIRE(grad && lr > 0.0, "bad arguments");
        lcc_alloc(ctx);
        Lcc &L = *ctx->lcc;
        hipStream_t s = S(stream);
        L.adam_step++;
        size_t off = 0;
        for (int l = 0; l < 3; ++l) {
            const size_t m = (size_t)L.wrows[l] * L.wcols[l];
            HIPCHK(hipMemcpyAsync(L.G[l], grad + off, m * sizeof(float), hipMemcpyDeviceToDevice, s));
            HIPCHK(lcc_adam(m, L.W[l], L.G[l], L.Mo[l], L.Vo[l], L.Wb[l], (float)lr, kAdamB1, kAdamB2, kAdamEps,
                            L.adam_step, s));
            off += m;
        }
    });
}

fr_status lcc_features_of(frpmg_ctx *ctx, const double *d1, float *rows_out, float *s_out, fr_stream stream) {
    return guarded(ctx, [&] {
        REQUIRE(d1 && rows_out && s_out, "null pointer");
        lcc_alloc(ctx);
        Lcc &L = *ctx->lcc;
        REQUIRE(L.scales_set, "scales not set");
        hipStream_t s = S(stream);
        HIPCHK(lcc_features(ctx, d1, L, L.Xf, L.Xb, L.srow, 0, s));
        HIPCHK(hipMemcpyAsync(rows_out, L.Xf, (size_t)ctx->mesh.Ne * L.nin_pad * sizeof(float),
                              hipMemcpyDeviceToDevice, s));
        HIPCHK(hipMemcpyAsync(s_out, L.srow, (size_t)ctx->mesh.Ne * sizeof(float), hipMemcpyDeviceToDevice, s));
    });
}

fr_status lcc_train(frpmg_ctx *ctx, const lcc_train_params *prm, lcc_train_stats *st, fr_stream stream) {
    lcc_train_stats local;
    lcc_train_stats *out = st ? st : &local;
    return guarded(ctx, [&] {
        REQUIRE(prm && prm->batch > 0 && prm->batch % 32 == 0, "batch must be a positive multiple of 32");
        REQUIRE(prm->epochs >= 1 && prm->lr > 0.0, "bad training parameters");
        REQUIRE(ctx->lcc && ctx->lcc->count >= 2 * prm->batch, "not enough harvested pairs");
        Lcc &L = *ctx->lcc;
        hipStream_t s = S(stream);
        std::memset(out, 0, sizeof(*out));
        HIPCHK(hipStreamSynchronize(s));
        const double t0 = now();
        if (prm->reinit) lcc_init_weights(ctx, prm->seed);
        const int B = prm->batch;
        lcc_train_buffers(ctx, B);
        const int nval = std::min(L.count - B, std::max(0, (int)(L.count * prm->holdout)));
        const int ntrain = L.count - nval;
        const int spe = ntrain / B;
        // batch index lists: at most count <= cap entries are written
        if (!L.perm || L.perm_cap < (size_t)L.cap) {
            dfree(L.perm);
            L.perm = talloc<int>(ctx, (size_t)L.cap);
            L.perm_cap = (size_t)L.cap;
        }
        auto val_loss = [&]() {
            const int nb = nval / B;
            if (nb == 0) return 0.0;
            std::vector<int> idx(nval);
            for (int i = 0; i < nval; ++i) idx[i] = ntrain + i;
            HIPCHK(hipMemcpy(L.perm, idx.data(), nval * sizeof(int), hipMemcpyHostToDevice));
            double acc = 0.0;
            for (int b = 0; b < nb; ++b) {
                HIPCHK(lcc_gather_batch(L, B, L.perm + (size_t)b * B, L.bX, L.bT, 0, s));
                lcc_forward_rows(ctx, B, L.bX, L.bH1, L.bH2, L.bY, s);
                HIPCHK(lcc_loss_grad(B, L.nout_pad, L.nout, L.bY, L.bT, L.bdY, L.lpart, L.lval, s));
                HIPCHK(hipMemcpyAsync(ctx->host_pinned, L.lval, sizeof(double), hipMemcpyDeviceToHost, s));
                HIPCHK(hipStreamSynchronize(s));
                acc += ctx->host_pinned[0];
            }
            return acc / nb;
        };
        out->val_loss_init = val_loss();
        std::mt19937_64 rng(prm->seed);
        std::vector<int> idx(ntrain);
        for (int i = 0; i < ntrain; ++i) idx[i] = i;
        for (int e = 0; e < prm->epochs; ++e) {
            std::shuffle(idx.begin(), idx.end(), rng);
            HIPCHK(hipMemcpy(L.perm, idx.data(), ntrain * sizeof(int), hipMemcpyHostToDevice));
            for (int b = 0; b < spe; ++b) {
                HIPCHK(lcc_gather_batch(L, B, L.perm + (size_t)b * B, L.bX, L.bT, 1, s));
                lcc_batch_grad(ctx, s);
                L.adam_step++;
                for (int l = 0; l < 3; ++l)
                    HIPCHK(lcc_adam((size_t)L.wrows[l] * L.wcols[l], L.W[l], L.G[l], L.Mo[l], L.Vo[l], L.Wb[l],
                                    (float)prm->lr, kAdamB1, kAdamB2, kAdamEps, L.adam_step, s));
                out->steps++;
                if (e == 0 && b == 0) {
                    HIPCHK(hipMemcpyAsync(ctx->host_pinned, L.lval, sizeof(double), hipMemcpyDeviceToHost, s));
                    HIPCHK(hipStreamSynchronize(s));
                    out->loss_first = ctx->host_pinned[0];
                }
            }
        }
        HIPCHK(hipMemcpyAsync(ctx->host_pinned, L.lval, sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        out->loss_last = ctx->host_pinned[0];
        out->val_loss = val_loss();
        L.weights_set = 1;
        HIPCHK(hipStreamSynchronize(s));
        out->t_train = now() - t0;
    });
}

// ---------------------------------------------------------------------------
// mixed polynomial degrees (p-adaptation)
// ---------------------------------------------------------------------------

fr_status fr_pa_hierarchy(const int *deg, int ne, int nlevels, int gap, int *out) {
    if (!deg || !out || ne < 1 || nlevels < 1 || nlevels > FR_MAX_LEVELS || (gap != 1 && gap != 2)) return FR_EINVAL;
    for (int k = 0; k < ne; ++k)
        if (deg[k] < 0 || deg[k] >= kMaxP) return FR_EINVAL;
    pa_nested(deg, ne, nlevels, gap, out);
    return FR_OK;
}

fr_status fr_set_degrees(frpmg_ctx *ctx, const int *host_deg, int gap) {
    return guarded(ctx, [&] {
        HIPCHK(hipDeviceSynchronize());
        clear_graphs(ctx);
        ctx->graph_epoch++;
        for (int l = 0; l < ctx->nlevels; ++l) {
            pa_free_level(ctx->lv[l]);
            ctx->lv[l].inv_prec = -1;
        }
        if (!host_deg) return;
        REQUIRE(gap == 1 || gap == 2, "order gap must be 1 or 2");
        REQUIRE(!ctx->mb, "MBNK smoothing is set up on this context");
        const int Ne = ctx->mesh.Ne;
        std::vector<int> deg((size_t)ctx->nlevels * Ne);
        for (int k = 0; k < Ne; ++k)
            REQUIRE(host_deg[k] >= 0 && host_deg[k] <= ctx->lv[0].p, "element degree outside [0, p of level 0]");
        pa_nested(host_deg, Ne, ctx->nlevels, gap, deg.data());
        for (int l = 0; l < ctx->nlevels; ++l) {
            const int mx = *std::max_element(deg.begin() + (size_t)l * Ne, deg.begin() + (size_t)(l + 1) * Ne);
            if (mx != ctx->lv[l].p) {
                char msg[160];
                std::snprintf(msg, sizeof msg,
                              "level %d of the nested hierarchy has largest degree %d but the context has p = %d", l, mx,
                              ctx->lv[l].p);
                ctx->err = msg;
                throw Fail{FR_EINVAL};
            }
        }
        ensure_pa_tables(ctx);
        for (int l = 0; l < ctx->nlevels; ++l) pa_build_level(ctx, l, deg.data() + (size_t)l * Ne);
        HIPCHK(hipDeviceSynchronize());
    });
}

fr_status fr_get_degrees(frpmg_ctx *ctx, int level, int *host_out) {
    return guarded(ctx, [&] {
        REQUIRE(level >= 0 && level < ctx->nlevels, "bad level");
        REQUIRE(host_out, "bad pointer");
        const Level &L = ctx->lv[level];
        for (int k = 0; k < ctx->mesh.Ne; ++k) host_out[k] = L.pa ? L.pa->Pk_host[k] - 1 : L.p;
    });
}

fr_status fr_pa_indicator(frpmg_ctx *ctx, int level, const double *dq, int var, double *eta, fr_stream stream) {
    return guarded(ctx, [&] {
        REQUIRE(level >= 0 && level < ctx->nlevels, "bad level");
        REQUIRE(dq && eta, "bad pointers");
        REQUIRE(var >= 0 && var < ctx->nv, "bad variable");
        const Level &L = ctx->lv[level];
        REQUIRE(L.pa, "the level has no degree map (fr_set_degrees)");
        for (int k = 0; k < ctx->mesh.Ne; ++k) REQUIRE(L.pa->Pk_host[k] >= 2, "the indicator needs degree >= 1");
        HIPCHK(pa_indicator(ctx, level, dq, var, eta, S(stream)));
    });
}

fr_status fr_pa_adapt(frpmg_ctx *ctx, const double *eta, const int *deg_in, int *deg_out, int p_min, int p_max,
                      double nu_max, double nu_min, fr_stream stream) {
    return guarded(ctx, [&] {
        REQUIRE(eta && deg_in && deg_out, "bad pointers");
        REQUIRE(p_min >= 0 && p_min <= p_max && p_max <= (ctx->dim == 2 ? 4 : 3), "bad degree range");
        REQUIRE(nu_min >= 0.0 && nu_min <= nu_max, "bad thresholds");
        HIPCHK(pa_adapt(ctx, eta, deg_in, deg_out, p_min, p_max, nu_max, nu_min, S(stream)));
    });
}

fr_status fr_pa_project(frpmg_ctx *ctx, const int *deg_from, int p_from, const double *x, const int *deg_to,
                        int p_to, double *y, fr_stream stream) {
    return guarded(ctx, [&] {
        REQUIRE(deg_from && deg_to && x && y && x != y, "bad pointers");
        const int pmax = ctx->dim == 2 ? 4 : 3;
        REQUIRE(p_from >= 0 && p_from <= pmax && p_to >= 0 && p_to <= pmax, "bad padded degree");
        ensure_pa_tables(ctx);
        const int NpF = ipow(p_from + 1, ctx->dim), NpT = ipow(p_to + 1, ctx->dim);
        HIPCHK(pa_project(ctx, deg_from, NpF, x, deg_to, NpT, y, S(stream)));
    });
}

}  // extern "C"
