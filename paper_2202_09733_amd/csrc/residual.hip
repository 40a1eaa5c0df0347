// FR residual R(q) for compressible Navier-Stokes on periodic tensor-product
// quads (2D) and hexes (3D), gfx950.
//
// R is the right-hand side of dq/dt = -div f (Sec. 2.1, Eq. (1)), discretised
// by flux reconstruction with Gauss-Legendre solution points, Huynh's
// DG-recovering corrections, flux-polynomial traces, the original Roe flux
// (no entropy fix, Sec. 4.2.1) and an LDG viscous flux (common solution from
// the +axis element, common viscous flux from the -axis element plus a
// penalty tau (q_R - q_L)).
//
// Three launches per evaluation, exchanging face data through L2/HBM:
//   1. k_traces : minus-end traces of the state along every axis      [dim][nv][NF][Ne]
//   2. k_faces  : corrected gradient per element, then the common flux on
//                 each element's + faces (Roe - LDG viscous)           [dim][nv][NF][Ne]
//   3. k_volume : corrected gradient again, pointwise fluxes, flux traces,
//                 divergence plus FR corrections -> R (or a fused output)
// Elements are processed EB at a time per workgroup, staged in LDS as
// [var][point][element] so that consecutive lanes touch consecutive elements
// (the HBM layout has the element index fastest, so global loads coalesce).
//
// State convention: every kernel evaluates at the deviation dq from the
// reference state, possibly plus a perturbation (SRC_AXPY: dq + alpha v;
// SRC_FDCOL: one block column perturbed in all elements of one parity
// colour).  Fluxes are formed as f(q) - f(q_inf) through identities exact in
// real arithmetic, so R(0) = 0 exactly.
#include "internal.hpp"

namespace frpmg {

namespace {

template <int DIM, int P>
struct Shape {
    static constexpr int NV = DIM + 2;
    static constexpr int NP = (DIM == 2) ? P * P : P * P * P;
    static constexpr int NF = (DIM == 2) ? P : P * P;
    static constexpr int EB = (256 / NP) > 0 ? (256 / NP) : 1;  // elements per workgroup
    static constexpr int NT = ((NP * EB + 63) / 64) * 64;      // threads per workgroup

    // local point on the line along axis a through face point f, position j
    __device__ __forceinline__ static int line(int a, int f, int j) {
        if (a == 0) return j + P * f;
        if (DIM == 2) return f + P * j;
        if (a == 1) return (f % P) + P * (j + P * (f / P));
        return f + P * P * j;
    }
    // face point index and position along axis a of local point i
    __device__ __forceinline__ static void split(int i, int a, int &f, int &ia) {
        if (a == 0) {
            ia = i % P;
            f = i / P;
        } else if (DIM == 2) {
            ia = i / P;
            f = i % P;
        } else if (a == 1) {
            ia = (i / P) % P;
            f = (i % P) + P * (i / (P * P));
        } else {
            ia = i / (P * P);
            f = i % (P * P);
        }
    }
};

__device__ __forceinline__ void coords(const MeshK &m, int k, int c[3]) {
    c[0] = k % m.n[0];
    int r = k / m.n[0];
    c[1] = r % m.n[1];
    c[2] = r / m.n[1];
}

__device__ __forceinline__ int neighbour(const MeshK &m, int k, int a, int s) {
    int c[3];
    coords(m, k, c);
    int x = c[a] + s;
    if (x < 0) x += m.n[a];
    if (x >= m.n[a]) x -= m.n[a];
    c[a] = x;
    return c[0] + m.n[0] * (c[1] + m.n[1] * c[2]);
}

__device__ __forceinline__ int colour_of(const MeshK &m, int k) {
    int c[3];
    coords(m, k, c);
    return (c[0] & 1) | ((c[1] & 1) << 1) | ((c[2] & 1) << 2);
}

__device__ __forceinline__ double sval(const Scal &s) { return s.p ? *s.p : s.v; }

struct SrcK {
    const double *dq;
    const double *v;
    Scal alpha;
    int colour, col, Np;
};

// Finite-difference step of one perturbed entry: 1e-7 max(1, |q_inf + dq|).
__device__ __forceinline__ double fd_step(double qinf_v, double dqv) {
    return 1e-7 * fmax(1.0, fabs(qinf_v + dqv));
}

template <int MODE>
__device__ __forceinline__ double load_state(const SrcK &s, const MeshK &m, const Phys &ph, int v, int i,
                                             int k, double alpha) {
    const size_t idx = ((size_t)v * s.Np + i) * m.Ne + k;
    double u = s.dq[idx];
    if (MODE == SRC_AXPY) u = fma(alpha, s.v[idx], u);
    if (MODE == SRC_FDCOL) {
        if (v * s.Np + i == s.col && colour_of(m, k) == s.colour) u = u + fd_step(ph.qinf[v], u);
    }
    return u;
}

// ---------------------------------------------------------------------------
// pointwise physics (deviation form)
// ---------------------------------------------------------------------------

template <int D>
struct PState {
    double rho, irho, E, p, dE, dp, drho;
    double u[D], du[D], dm[D];
};

template <int D>
__device__ __forceinline__ void pstate(const Phys &ph, const double *dq, PState<D> &s) {
    s.drho = dq[0];
    s.rho = ph.qinf[0] + s.drho;
    s.irho = 1.0 / s.rho;
    double two_dk = 0.0;
#pragma unroll
    for (int b = 0; b < D; ++b) {
        s.dm[b] = dq[1 + b];
        s.u[b] = (ph.qinf[1 + b] + s.dm[b]) * s.irho;
        s.du[b] = (s.dm[b] - ph.uinf[b] * s.drho) * s.irho;  // u - u_inf
        two_dk += s.dm[b] * s.u[b] + ph.qinf[1 + b] * s.du[b];
    }
    s.dE = dq[D + 1];
    s.E = ph.qinf[D + 1] + s.dE;
    s.dp = (ph.gam - 1.0) * (s.dE - 0.5 * two_dk);
    s.p = ph.pinf + s.dp;
}

// f^I_a(q) - f^I_a(q_inf)
template <int D>
__device__ __forceinline__ void inviscid_dev(const Phys &ph, int a, const PState<D> &s, double *F) {
    F[0] = s.dm[a];
#pragma unroll
    for (int b = 0; b < D; ++b) F[1 + b] = s.dm[a] * s.u[b] + ph.qinf[1 + a] * s.du[b] + (a == b ? s.dp : 0.0);
    F[D + 1] = s.du[a] * (s.E + s.p) + ph.uinf[a] * (s.dE + s.dp);
}

// viscous flux along a from conservative gradients g[c][v]
template <int D>
__device__ __forceinline__ void viscous(const Phys &ph, int a, const PState<D> &s, const double (&g)[D][D + 2],
                                        double *F) {
    double gu[D][D];  // gu[b][c] = d u_b / d x_c
    double ge[D];
    const double et = s.E * s.irho;
#pragma unroll
    for (int c = 0; c < D; ++c) {
        double kin = 0.0;
#pragma unroll
        for (int b = 0; b < D; ++b) {
            gu[b][c] = (g[c][1 + b] - s.u[b] * g[c][0]) * s.irho;
            kin += s.u[b] * gu[b][c];
        }
        ge[c] = (g[c][D + 1] - et * g[c][0]) * s.irho - kin;
    }
    double div = 0.0;
#pragma unroll
    for (int b = 0; b < D; ++b) div += gu[b][b];
    F[0] = 0.0;
    double work = 0.0;
#pragma unroll
    for (int b = 0; b < D; ++b) {
        double t = ph.mu * (gu[a][b] + gu[b][a]);
        if (a == b) t -= (2.0 / 3.0) * ph.mu * div;
        F[1 + b] = t;
        work += s.u[b] * t;
    }
    F[D + 1] = work + (ph.mu * ph.gam / ph.Pr) * ge[a];
}

// Roe flux along a, deviation form, no entropy fix.
template <int D>
__device__ __forceinline__ void roe(const Phys &ph, int a, const double *qL, const double *qR, double *F) {
    PState<D> L, R;
    pstate<D>(ph, qL, L);
    pstate<D>(ph, qR, R);
    double FL[D + 2], FR[D + 2];
    inviscid_dev<D>(ph, a, L, FL);
    inviscid_dev<D>(ph, a, R, FR);
    const double sl = sqrt(L.rho), sr = sqrt(R.rho);
    const double iw = 1.0 / (sl + sr);
    const double rt = sl * sr;
    double ut[D], q2 = 0.0;
#pragma unroll
    for (int b = 0; b < D; ++b) {
        ut[b] = (sl * L.u[b] + sr * R.u[b]) * iw;
        q2 += ut[b] * ut[b];
    }
    const double Ht = (sl * (L.E + L.p) * L.irho + sr * (R.E + R.p) * R.irho) * iw;
    const double c2 = (ph.gam - 1.0) * (Ht - 0.5 * q2);
    const double ct = sqrt(c2);
    const double ic2 = 1.0 / c2;
    const double un = ut[a];
    const double jr = R.drho - L.drho;
    const double jp = R.dp - L.dp;
    double ju[D];
#pragma unroll
    for (int b = 0; b < D; ++b) ju[b] = R.du[b] - L.du[b];
    const double jun = ju[a];
    const double w1 = fabs(un - ct) * 0.5 * (jp - rt * ct * jun) * ic2;  // |l1| alpha1
    const double w3 = fabs(un + ct) * 0.5 * (jp + rt * ct * jun) * ic2;  // |l3| alpha3
    const double w2 = fabs(un) * (jr - jp * ic2);                       // |l2| alpha2
    const double ws = fabs(un) * rt;                                    // shear waves
    double dis[D + 2];
    dis[0] = w1 + w2 + w3;
    double utju = 0.0;
#pragma unroll
    for (int b = 0; b < D; ++b) {
        const double nb = (a == b) ? 1.0 : 0.0;
        dis[1 + b] = w1 * (ut[b] - ct * nb) + w2 * ut[b] + w3 * (ut[b] + ct * nb) + ws * (ju[b] - nb * jun);
        utju += ut[b] * ju[b];
    }
    dis[D + 1] = w1 * (Ht - un * ct) + w2 * 0.5 * q2 + w3 * (Ht + un * ct) + ws * (utju - un * jun);
#pragma unroll
    for (int v = 0; v < D + 2; ++v) F[v] = 0.5 * (FL[v] + FR[v]) - 0.5 * dis[v];
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

template <int DIM, int P, int MODE>
__global__ void __launch_bounds__(256) k_traces(MeshK m, SrcK src, Ops1D ops, Phys ph, double *__restrict__ Tm) {
    using S = Shape<DIM, P>;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m.Ne) return;
    const int a = blockIdx.y / S::NF;
    const int f = blockIdx.y % S::NF;
    const double alpha = (MODE == SRC_AXPY) ? sval(src.alpha) : 0.0;
#pragma unroll
    for (int v = 0; v < S::NV; ++v) {
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < P; ++j) s += ops.bm[j] * load_state<MODE>(src, m, ph, v, S::line(a, f, j), k, alpha);
        Tm[((size_t)(a * S::NV + v) * S::NF + f) * m.Ne + k] = s;
    }
}

// Shared staging of a workgroup's elements: state, neighbour traces, 2/h.
template <int DIM, int P, int MODE>
__device__ __forceinline__ void stage_elements(const MeshK &m, const SrcK &src, const Phys &ph,
                                               const double *__restrict__ Tm, int k0, int ne, double *s_u,
                                               double *s_t, double *s_ih, double alpha) {
    using S = Shape<DIM, P>;
    constexpr int EB = S::EB;
    for (int t = threadIdx.x; t < S::NV * S::NP * EB; t += blockDim.x) {
        const int e = t % EB, vi = t / EB;
        const int v = vi / S::NP, i = vi % S::NP;
        s_u[t] = (e < ne) ? load_state<MODE>(src, m, ph, v, i, k0 + e, alpha) : 0.0;
    }
    for (int t = threadIdx.x; t < DIM * S::NV * S::NF * EB; t += blockDim.x) {
        const int e = t % EB;
        int r = t / EB;
        const int f = r % S::NF;
        r /= S::NF;
        const int v = r % S::NV, a = r / S::NV;
        double val = 0.0;
        if (e < ne) {
            const int kn = neighbour(m, k0 + e, a, +1);
            val = Tm[((size_t)(a * S::NV + v) * S::NF + f) * m.Ne + kn];
        }
        s_t[t] = val;
    }
    for (int t = threadIdx.x; t < DIM * EB; t += blockDim.x) {
        const int e = t % EB, a = t / EB;
        double val = 0.0;
        if (e < ne) {
            int c[3];
            coords(m, k0 + e, c);
            val = m.inv2h[a][c[a]];
        }
        s_ih[t] = val;
    }
}

// Corrected gradient at one point of one staged element (the common solution
// is the +axis element's trace, so only the + end carries a correction).
template <int DIM, int P>
__device__ __forceinline__ void gradient_point(const Ops1D &ops, const double *s_u, const double *s_t,
                                               const double *s_ih, int e, int i, double (&g)[DIM][DIM + 2]) {
    using S = Shape<DIM, P>;
    constexpr int EB = S::EB;
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        int f, ic;
        S::split(i, c, f, ic);
        const double ih = s_ih[c * EB + e];
#pragma unroll
        for (int v = 0; v < S::NV; ++v) {
            double d = 0.0, tp = 0.0;
#pragma unroll
            for (int j = 0; j < P; ++j) {
                const double q = s_u[(v * S::NP + S::line(c, f, j)) * EB + e];
                d += ops.D[ic][j] * q;
                tp += ops.bp[j] * q;
            }
            d += (s_t[((c * S::NV + v) * S::NF + f) * EB + e] - tp) * ops.gRd[ic];
            g[c][v] = ih * d;
        }
    }
}

template <int DIM, int P, int MODE>
__global__ void __launch_bounds__((Shape<DIM, P>::NT)) k_faces(MeshK m, SrcK src, Ops1D ops_in, Phys ph,
                                                            const double *__restrict__ Tm,
                                                            double *__restrict__ Fs) {
    using S = Shape<DIM, P>;
    constexpr int EB = S::EB, NV = S::NV, NP = S::NP, NF = S::NF;
    __shared__ Ops1D ops;
    __shared__ double s_u[NV * NP * EB];
    __shared__ double s_t[DIM * NV * NF * EB];
    __shared__ double s_g[DIM * NV * NP * EB];
    __shared__ double s_ih[DIM * EB];
    if (threadIdx.x == 0) ops = ops_in;
    const int k0 = blockIdx.x * EB;
    const int ne = min(EB, m.Ne - k0);
    const double alpha = (MODE == SRC_AXPY) ? sval(src.alpha) : 0.0;
    stage_elements<DIM, P, MODE>(m, src, ph, Tm, k0, ne, s_u, s_t, s_ih, alpha);
    __syncthreads();
    {
        const int t = threadIdx.x;
        const int e = t % EB, i = t / EB;
        if (t < NP * EB && e < ne) {
            double g[DIM][DIM + 2];
            gradient_point<DIM, P>(ops, s_u, s_t, s_ih, e, i, g);
#pragma unroll
            for (int c = 0; c < DIM; ++c)
#pragma unroll
                for (int v = 0; v < NV; ++v) s_g[((c * NV + v) * NP + i) * EB + e] = g[c][v];
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < DIM * NF * EB; t += blockDim.x) {
        const int e = t % EB;
        const int r = t / EB;
        const int f = r % NF, a = r / NF;
        if (e >= ne) continue;
        double qL[NV], qR[NV], gL[DIM][DIM + 2];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            double s = 0.0;
#pragma unroll
            for (int j = 0; j < P; ++j) s += ops.bp[j] * s_u[(v * NP + S::line(a, f, j)) * EB + e];
            qL[v] = s;
            qR[v] = s_t[((a * NV + v) * NF + f) * EB + e];
        }
#pragma unroll
        for (int c = 0; c < DIM; ++c)
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                double s = 0.0;
#pragma unroll
                for (int j = 0; j < P; ++j) s += ops.bp[j] * s_g[((c * NV + v) * NP + S::line(a, f, j)) * EB + e];
                gL[c][v] = s;
            }
        double Fr[NV], Fv[NV];
        roe<DIM>(ph, a, qL, qR, Fr);
        PState<DIM> sL;
        pstate<DIM>(ph, qL, sL);
        viscous<DIM>(ph, a, sL, gL, Fv);
#pragma unroll
        for (int v = 0; v < NV; ++v)
            Fs[((size_t)(a * NV + v) * NF + f) * m.Ne + k0 + e] = Fr[v] - (Fv[v] + ph.tau * (qR[v] - qL[v]));
    }
}

struct OutK {
    double *r;
    const double *r0;
    const double *x;
    const double *vdir;
    double sigma;
    double *blocks;
    int nb;
};

template <int DIM, int P, int MODE, int OUT>
__global__ void __launch_bounds__((Shape<DIM, P>::NT)) k_volume(MeshK m, SrcK src, Ops1D ops_in, Phys ph,
                                                             const double *__restrict__ Tm,
                                                             const double *__restrict__ Fs, OutK o) {
    using S = Shape<DIM, P>;
    constexpr int EB = S::EB, NV = S::NV, NP = S::NP, NF = S::NF;
    __shared__ Ops1D ops;
    __shared__ double s_u[NV * NP * EB];
    __shared__ double s_t[DIM * NV * NF * EB];
    __shared__ double s_g[DIM * NV * NP * EB];  // pointwise fluxes
    __shared__ double s_fp[DIM * NV * NF * EB];
    __shared__ double s_fm[DIM * NV * NF * EB];
    __shared__ double s_ih[DIM * EB];
    if (threadIdx.x == 0) ops = ops_in;
    const int k0 = blockIdx.x * EB;
    const int ne = min(EB, m.Ne - k0);
    const double alpha = (MODE == SRC_AXPY) ? sval(src.alpha) : 0.0;
    stage_elements<DIM, P, MODE>(m, src, ph, Tm, k0, ne, s_u, s_t, s_ih, alpha);
    for (int t = threadIdx.x; t < DIM * NV * NF * EB; t += blockDim.x) {
        const int e = t % EB;
        const int r = t / EB;  // (a*NV + v)*NF + f
        const int a = r / (NV * NF);
        double vp = 0.0, vm = 0.0;
        if (e < ne) {
            const int k = k0 + e;
            vp = Fs[(size_t)r * m.Ne + k];
            vm = Fs[(size_t)r * m.Ne + neighbour(m, k, a, -1)];
        }
        s_fp[t] = vp;
        s_fm[t] = vm;
    }
    __syncthreads();
    const int t = threadIdx.x;
    const int e = t % EB, i = t / EB;
    // EJ columns: only elements of the perturbed colour produce output, and
    // their residual needs no other element's pointwise fluxes
    const bool active = (t < NP * EB) && (e < ne) && (OUT != OUT_EJCOL || colour_of(m, k0 + e) == src.colour);
    double g[DIM][DIM + 2];
    if (active) gradient_point<DIM, P>(ops, s_u, s_t, s_ih, e, i, g);
    // the gradient stays in registers; s_g now receives the pointwise fluxes
    if (active) {
        double q[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) q[v] = s_u[(v * NP + i) * EB + e];
        PState<DIM> st;
        pstate<DIM>(ph, q, st);
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            double FI[NV], FV[NV];
            inviscid_dev<DIM>(ph, a, st, FI);
            viscous<DIM>(ph, a, st, g, FV);
#pragma unroll
            for (int v = 0; v < NV; ++v) s_g[((a * NV + v) * NP + i) * EB + e] = FI[v] - FV[v];
        }
    }
    __syncthreads();
    if (!active) return;
    const int k = k0 + e;
    double hact = 1.0;
    bool write_col = true;
    if (OUT == OUT_EJCOL) {
        write_col = (colour_of(m, k) == src.colour);
        const size_t jidx = (size_t)src.col * m.Ne + k;
        const int jv = src.col / NP;
        const double base = src.dq[jidx];
        hact = (base + fd_step(ph.qinf[jv], base)) - base;
        if (!write_col) return;
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        double acc = 0.0;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            int f, ia;
            S::split(i, a, f, ia);
            double d = 0.0, fm = 0.0, fp = 0.0;
#pragma unroll
            for (int j = 0; j < P; ++j) {
                const double x = s_g[((a * NV + v) * NP + S::line(a, f, j)) * EB + e];
                d += ops.D[ia][j] * x;
                fm += ops.bm[j] * x;
                fp += ops.bp[j] * x;
            }
            const int fi = ((a * NV + v) * NF + f) * EB + e;
            d += (s_fm[fi] - fm) * ops.gLd[ia] + (s_fp[fi] - fp) * ops.gRd[ia];
            acc += s_ih[a * EB + e] * d;
        }
        const double R = -acc;
        const size_t idx = ((size_t)v * NP + i) * m.Ne + k;
        if (OUT == OUT_R) {
            o.r[idx] = R;
        } else if (OUT == OUT_LIN) {
            double val = o.sigma * o.vdir[idx] - (R - o.r0[idx]) / alpha;
            if (o.x) val -= o.x[idx];
            o.r[idx] = val;
        } else {
            const int row = v * NP + i;
            double val = -(R - o.r0[idx]) / hact;
            if (row == src.col) val += o.sigma;
            o.blocks[(size_t)k * o.nb * o.nb + (size_t)src.col * o.nb + row] = val;
        }
    }
}

template <int DIM, int P, int MODE, int OUT>
hipError_t run(const frpmg_ctx *ctx, const Level &L, const ResidualArgs &a, hipStream_t s) {
    using S = Shape<DIM, P>;
    const MeshK &m = ctx->mesh;
    SrcK src{a.dq, a.v, a.alpha, a.colour, a.col, S::NP};
    dim3 g0((m.Ne + 255) / 256, DIM * S::NF);
    hipLaunchKernelGGL((k_traces<DIM, P, MODE>), g0, dim3(256), 0, s, m, src, L.ops, ctx->phys, L.Tm);
    dim3 g1((m.Ne + S::EB - 1) / S::EB);
    hipLaunchKernelGGL((k_faces<DIM, P, MODE>), g1, dim3(S::NT), 0, s, m, src, L.ops, ctx->phys, L.Tm, L.Fs);
    OutK o{a.r, a.r0, a.x, a.v, a.sigma, a.blocks, L.nb};
    hipLaunchKernelGGL((k_volume<DIM, P, MODE, OUT>), g1, dim3(S::NT), 0, s, m, src, L.ops, ctx->phys, L.Tm,
                       L.Fs, o);
    return hipGetLastError();
}

template <int DIM, int P>
hipError_t dispatch_modes(const frpmg_ctx *ctx, const Level &L, const ResidualArgs &a, hipStream_t s) {
    if (a.src == SRC_PLAIN && a.out == OUT_R) return run<DIM, P, SRC_PLAIN, OUT_R>(ctx, L, a, s);
    if (a.src == SRC_AXPY && a.out == OUT_R) return run<DIM, P, SRC_AXPY, OUT_R>(ctx, L, a, s);
    if (a.src == SRC_AXPY && a.out == OUT_LIN) return run<DIM, P, SRC_AXPY, OUT_LIN>(ctx, L, a, s);
    if (a.src == SRC_FDCOL && a.out == OUT_EJCOL) return run<DIM, P, SRC_FDCOL, OUT_EJCOL>(ctx, L, a, s);
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_residual(const frpmg_ctx *ctx, int level, const ResidualArgs &a, hipStream_t s) {
    const Level &L = ctx->lv[level];
    if (ctx->dim == 2) {
        switch (L.P) {
            case 2: return dispatch_modes<2, 2>(ctx, L, a, s);
            case 3: return dispatch_modes<2, 3>(ctx, L, a, s);
            case 4: return dispatch_modes<2, 4>(ctx, L, a, s);
            case 5: return dispatch_modes<2, 5>(ctx, L, a, s);
        }
    } else {
        switch (L.P) {
            case 2: return dispatch_modes<3, 2>(ctx, L, a, s);
            case 3: return dispatch_modes<3, 3>(ctx, L, a, s);
            case 4: return dispatch_modes<3, 4>(ctx, L, a, s);
        }
    }
    return hipErrorInvalidValue;
}

}  // namespace frpmg
