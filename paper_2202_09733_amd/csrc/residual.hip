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
// Two launches per evaluation, exchanging face data through L2/HBM:
//   1. k_faces  : the common flux on each element's + faces, and the state
//                 jump q* - q+ there (q* = the + neighbour's minus-end trace,
//                 formed from the neighbour's state while staging).  The corrected
//                 gradient is needed there only as a + face trace, which is
//                 formed by sum factorisation from the state's face traces
//                 (normal part: a 1D row operator; tangential parts: D along
//                 the face plus the + end value of the neighbouring faces'
//                 jumps), so no volume gradient is formed.   2 x [dim][nv][NF][Ne]
//   2. k_volume : corrected gradient (registers), pointwise fluxes one
//                 direction at a time through LDS, divergence plus FR
//                 corrections -> R (or a fused output).
// Face quantities that every solution point on a line needs (state jumps
// q* - q+, flux jumps F* - f-/+) are formed once per face point.
// Elements are processed EB at a time per workgroup, staged in LDS as
// [var][point][element] so that consecutive lanes touch consecutive elements
// (the HBM layout has the element index fastest, so global loads coalesce).
//
// State convention: every kernel evaluates at the deviation dq from the
// reference state, possibly plus a direction (SRC_AXPY: dq + alpha v).
// Fluxes are formed as f(q) - f(q_inf) through identities exact in real
// arithmetic, so R(0) = 0 exactly.
//
// The element-Jacobi blocks are formed element-locally (k_ej_form, below).
#include <algorithm>
#include <type_traits>

#include "internal.hpp"

namespace frpmg {

namespace {

constexpr int round64(int n) { return ((n + 63) / 64) * 64; }

template <int DIM, int P>
struct Shape {
    static constexpr int NV = DIM + 2;
    static constexpr int NP = (DIM == 2) ? P * P : P * P * P;
    static constexpr int NF = (DIM == 2) ? P : P * P;
    // volume kernel: one lane per (element, point); one point per element
    // (p = 0) takes 64 elements per workgroup to bound the LDS staging
    static constexpr int EB = (P == 1) ? 64 : ((256 / NP) > 0 ? (256 / NP) : 1);
    static constexpr int NT = round64(NP * EB);
    static constexpr int NTV = (DIM == 2) ? 2 * NT : NT;  // volume kernel threads (2D: two lanes per point)
    // face kernel: one lane per (element, + face point), the lanes of each
    // flux direction in whole wavefronts (LPA per axis), so that no
    // wavefront runs two directions' flux code one after the other.  2D
    // fills half of each wavefront (32 lanes per direction): the kernel is
    // latency-bound there, and twice the workgroups spread it over more CUs
    // (config-2 residual 19.3 -> 17.5 us)
    static constexpr int EBF = (DIM == 2) ? (NF >= 32 ? 1 : 32 / NF) : (NF >= 64 ? 1 : 64 / NF);
    static constexpr int LPA = round64(NF * EBF);
    static constexpr int NTF = DIM * LPA;
    static constexpr bool SPLIT = (DIM == 2);        // face kernel: viscous and Roe parts in separate wavefronts
    static constexpr int NTF2 = SPLIT ? 2 * NTF : NTF;  // face kernel threads

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
    // index on the face normal to axis a of the point with coordinates x
    // (the remaining coordinates in increasing axis order, first fastest)
    __device__ __forceinline__ static int face_index(int a, const int (&x)[3]) {
        if (DIM == 2) return a == 0 ? x[1] : x[0];
        if (a == 0) return x[1] + P * x[2];
        if (a == 1) return x[0] + P * x[2];
        return x[0] + P * x[1];
    }
    __device__ __forceinline__ static void face_coords(int a, int f, int (&x)[3]) {
        x[0] = x[1] = x[2] = 0;
        if (DIM == 2) {
            x[a == 0 ? 1 : 0] = f;
        } else if (a == 0) {
            x[1] = f % P;
            x[2] = f / P;
        } else if (a == 1) {
            x[0] = f % P;
            x[2] = f / P;
        } else {
            x[0] = f % P;
            x[1] = f / P;
        }
    }
};

struct SrcK {
    const double *dq;
    const double *v;
    Scal alpha;
    int Np;
};

template <int MODE>
__device__ __forceinline__ double load_state(const SrcK &s, const MeshK &m, int v, int i, int k, double alpha) {
    const size_t idx = ((size_t)v * s.Np + i) * m.Ne + k;
    double u = s.dq[idx];
    if (MODE == SRC_AXPY) u = fma(alpha, s.v[idx], u);
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


// Gradients of the primitive variables at one point from the conservative
// gradients g[c][v]: gu[b][c] = d u_b / d x_c, ge[c] = d e / d x_c (e the
// specific internal energy), div = div u.  Shared by every flux direction.
template <int D>
struct VGrad {
    double gu[D][D];
    double ge[D];
    double div;
};

template <int D>
__device__ __forceinline__ void vgrad(const PState<D> &s, const double (&g)[D][D + 2], VGrad<D> &w) {
    const double et = s.E * s.irho;
#pragma unroll
    for (int c = 0; c < D; ++c) {
        double kin = 0.0;
#pragma unroll
        for (int b = 0; b < D; ++b) {
            w.gu[b][c] = (g[c][1 + b] - s.u[b] * g[c][0]) * s.irho;
            kin += s.u[b] * w.gu[b][c];
        }
        w.ge[c] = (g[c][D + 1] - et * g[c][0]) * s.irho - kin;
    }
    double div = 0.0;
#pragma unroll
    for (int b = 0; b < D; ++b) div += w.gu[b][b];
    w.div = div;
}

// viscous flux along a (constant mu, Stokes hypothesis, Fourier heat flux)
template <int D>
__device__ __forceinline__ void viscous_dir(const Phys &ph, int a, const PState<D> &s, const VGrad<D> &w,
                                            double *F) {
    F[0] = 0.0;
    double work = 0.0;
#pragma unroll
    for (int b = 0; b < D; ++b) {
        double t = ph.mu * (w.gu[a][b] + w.gu[b][a]);
        if (a == b) t -= (2.0 / 3.0) * ph.mu * w.div;
        F[1 + b] = t;
        work += s.u[b] * t;
    }
    F[D + 1] = work + (ph.mu * ph.gam / ph.Pr) * w.ge[a];
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

// Index into an LDS array whose trailing dimension is the workgroup slot
// with stride SL (SL = 0: one copy shared by every slot).
template <int SL>
__device__ __forceinline__ int sidx(int base, int e) {
    return SL ? base * SL + e : base;
}

// Stage the EB elements k0 .. k0 + ne - 1: the state [v][i][e], face data
// on the + faces [a][v][f][e] and 2/h per axis [a][e].  TRACE: the face data
// is q*, the + neighbour's minus-end trace, formed here from the neighbour's
// state; otherwise it is read from Fd ([a][v][f][Ne], written by k_faces).
template <int DIM, int P, int MODE, int EB, bool TRACE>
__device__ __forceinline__ void stage_state(const MeshK &m, const SrcK &src, const Ops1D &ops,
                                            const double *__restrict__ Fd, int k0, int ne, double *s_u,
                                            double *s_t, double *s_ih, double alpha) {
    using S = Shape<DIM, P>;
    for (int t = threadIdx.x; t < S::NV * S::NP * EB; t += blockDim.x) {
        const int e = t % EB, vi = t / EB;
        s_u[t] = (e < ne) ? load_state<MODE>(src, m, vi / S::NP, vi % S::NP, k0 + e, alpha) : 0.0;
    }
    for (int t = threadIdx.x; t < DIM * S::NV * S::NF * EB; t += blockDim.x) {
        const int e = t % EB;
        const int r = t / EB;  // (a * NV + v) * NF + f
        double val = 0.0;
        if (e < ne) {
            if (TRACE) {
                const int f = r % S::NF;
                const int v = (r / S::NF) % S::NV, a = r / (S::NF * S::NV);
                const int kn = neighbour(m, k0 + e, a, +1);
#pragma unroll
                for (int j = 0; j < P; ++j) val += ops.bm[j] * load_state<MODE>(src, m, v, S::line(a, f, j), kn, alpha);
            } else {
                val = Fd[(size_t)r * m.Ne + k0 + e];
            }
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

// State and gradient traces at one point of the + face normal to A of slot
// e.  s_u [v][i][slot], s_qp = own + traces [a][v][f][slot]; s_t = q* on the
// + faces and s_ih = 2/h [a], both with slot stride TS (0: shared).  The
// gradient trace is formed by sum factorisation: the normal component from
// the row operator dnp = l(+1)^T D and the + end value cgp of the right
// correction; each tangential component from D along the face applied to
// the + traces plus the + end value of the jumps on the neighbouring face.
// Sn receives the normal component's D part before the correction.
template <int DIM, int P, int A, int EB, int TS>
__device__ __forceinline__ void plus_face_state(const Ops1D &ops, const double *s_u, const double *s_t,
                                                const double *s_qp, const double *s_ih, int e, int f,
                                                double (&qL)[DIM + 2], double (&qR)[DIM + 2],
                                                double (&g)[DIM][DIM + 2], double (&Sn)[DIM + 2]) {
    using S = Shape<DIM, P>;
    constexpr int NV = S::NV, NP = S::NP, NF = S::NF;
    int x[3];
    S::face_coords(A, f, x);
    const double ihA = s_ih[sidx<TS>(A, e)];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const int fb = (A * NV + v) * NF + f;
        qL[v] = s_qp[fb * EB + e];
        qR[v] = s_t[sidx<TS>(fb, e)];
        double d = 0.0;
#pragma unroll
        for (int j = 0; j < P; ++j) d += ops.dnp[j] * s_u[(v * NP + S::line(A, f, j)) * EB + e];
        Sn[v] = d;
        d += (qR[v] - qL[v]) * ops.cgp;
        g[A][v] = ihA * d;
    }
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        if (c == A) continue;
        const int ic = x[c];
        const double ihc = s_ih[sidx<TS>(c, e)];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            double d = 0.0;
#pragma unroll
            for (int l = 0; l < P; ++l) {
                int y[3] = {x[0], x[1], x[2]};
                y[c] = l;
                d += ops.D[ic][l] * s_qp[((A * NV + v) * NF + S::face_index(A, y)) * EB + e];
            }
            double jt = 0.0;
#pragma unroll
            for (int i = 0; i < P; ++i) {
                int y[3] = {x[0], x[1], x[2]};
                y[A] = i;
                const int fj = (c * NV + v) * NF + S::face_index(c, y);
                jt += ops.bp[i] * (s_t[sidx<TS>(fj, e)] - s_qp[fj * EB + e]);
            }
            d += jt * ops.gRd[ic];
            g[c][v] = ihc * d;
        }
    }
}

// Common flux along A from the two states and the -axis side's gradient:
// F* = Roe(qL, qR) - (f^V(qL, g) + tau (qR - qL)).
template <int DIM, int A>
__device__ __forceinline__ void common_flux(const Phys &ph, const double (&qL)[DIM + 2], const double (&qR)[DIM + 2],
                                            const double (&g)[DIM][DIM + 2], double (&F)[DIM + 2]) {
    constexpr int NV = DIM + 2;
    double Fv[NV], Fr[NV];
    {
        PState<DIM> sL;
        pstate<DIM>(ph, qL, sL);
        VGrad<DIM> w;
        vgrad<DIM>(sL, g, w);
        viscous_dir<DIM>(ph, A, sL, w, Fv);
    }
    roe<DIM>(ph, A, qL, qR, Fr);
#pragma unroll
    for (int v = 0; v < NV; ++v) F[v] = Fr[v] - (Fv[v] + ph.tau * (qR[v] - qL[v]));
}

// Face data of the linearisation point kept for the element-local EJ
// formation: per + face of its owner, q* there, the owner's + trace, the D
// part of the normal gradient and the tangential gradient components.
struct FaceSave {
    double *Qs;  // q*, the + neighbour's minus trace [a][v][f][Ne]
    double *Qp;  // [a][v][f][Ne]
    double *Sn;  // [a][v][f][Ne]
    double *Gt;  // [a][c'][v][f][Ne], c' over the axes other than a in increasing order
};

// Common flux on one + face point; also writes the state jump q* - q+ there
// (Jp), which the volume kernel needs, and the saved base data.
template <int DIM, int P, int A, int EB, bool SAVE>
__device__ __forceinline__ void face_flux(const MeshK &m, const Ops1D &ops, const Phys &ph, const double *s_u,
                                          const double *s_t, const double *s_qp, const double *s_ih, int e,
                                          int f, int k, double *__restrict__ Fs, double *__restrict__ Jp,
                                          const FaceSave &sv) {
    using S = Shape<DIM, P>;
    constexpr int NV = S::NV, NF = S::NF;
    double qL[NV], qR[NV], g[DIM][NV], Sn[NV], F[NV];
    plus_face_state<DIM, P, A, EB, EB>(ops, s_u, s_t, s_qp, s_ih, e, f, qL, qR, g, Sn);
#pragma unroll
    for (int v = 0; v < NV; ++v) Jp[((size_t)(A * NV + v) * NF + f) * m.Ne + k] = qR[v] - qL[v];
    if (SAVE) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const size_t o = ((size_t)(A * NV + v) * NF + f) * m.Ne + k;
            sv.Qs[o] = qR[v];
            sv.Qp[o] = qL[v];
            sv.Sn[o] = Sn[v];
#pragma unroll
            for (int c = 0; c < DIM; ++c) {
                if (c == A) continue;
                const int cc = c < A ? c : c - 1;
                sv.Gt[((size_t)((A * (DIM - 1) + cc) * NV + v) * NF + f) * m.Ne + k] = g[c][v];
            }
        }
    }
    common_flux<DIM, A>(ph, qL, qR, g, F);
#pragma unroll
    for (int v = 0; v < NV; ++v) Fs[((size_t)(A * NV + v) * NF + f) * m.Ne + k] = F[v];
}

// Face kernel: one lane per (element, + face point), the lanes of each flux
// direction in whole wavefronts.  In 2D each direction has two wavefronts:
// one forms the gradient trace and the viscous part of the common flux (and
// writes the state jumps and saved face data), the other the Roe flux from
// the two traces; they meet through LDS after one barrier, with
// common_flux()'s arithmetic in the same order.  Each wavefront's chain of
// dependent arithmetic is then about half of the whole common flux, which
// pays on the latency-bound 2D meshes (64x64 p = 4: 8.7 -> 7.7 us, 10.0 ->
// 9.2 us linearised).  In 3D the kernel is bound by throughput and the split
// (six wavefronts per workgroup, the pressure point spilling at 128
// registers) took 178 us against 122: there one lane computes the whole
// common flux (face_flux()), at most 128 VGPRs (four waves per SIMD; the 3D
// face flux otherwise takes ~131).
template <int DIM, int P, int MODE, bool SAVE>
__global__ void __launch_bounds__((Shape<DIM, P>::NTF2)) __attribute__((amdgpu_waves_per_eu(4, 8)))
k_faces(MeshK m, SrcK src, Ops1D ops_in, Phys ph, double *__restrict__ Jp, double *__restrict__ Fs, FaceSave sv) {
    using S = Shape<DIM, P>;
    constexpr int EB = S::EBF, NV = S::NV, NP = S::NP, NF = S::NF;
    constexpr int NFACE = DIM * NV * NF * EB;
    __shared__ Ops1D ops;
    __shared__ double s_u[NV * NP * EB];
    __shared__ double s_t[NFACE];   // q* on the + faces (the + neighbour's minus trace)
    __shared__ double s_qp[NFACE];  // q+ (own plus trace)
    constexpr bool SPLIT = Shape<DIM, P>::SPLIT;
    __shared__ double s_x[SPLIT ? NFACE : 1];  // f^V(q+, g) + tau (q* - q+) from the viscous wavefronts
    __shared__ double s_ih[DIM * EB];
    if (threadIdx.x == 0) ops = ops_in;
    const int k0 = xcd_block(blockIdx.x, gridDim.x) * EB;
    const int ne = min(EB, m.Ne - k0);
    const double alpha = (MODE == SRC_AXPY) ? sval(src.alpha) : 0.0;
    stage_state<DIM, P, MODE, EB, true>(m, src, ops_in, nullptr, k0, ne, s_u, s_t, s_ih, alpha);
    __syncthreads();
    for (int t = threadIdx.x; t < NFACE; t += blockDim.x) {
        const int e = t % EB;
        int r = t / EB;
        const int f = r % NF;
        r /= NF;
        const int v = r % NV, a = r / NV;
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < P; ++j) s += ops.bp[j] * s_u[(v * NP + S::line(a, f, j)) * EB + e];
        s_qp[t] = s;
    }
    __syncthreads();
    if constexpr (!SPLIT) {
        // one face point per lane; the direction is uniform over each wavefront
        const int a = __builtin_amdgcn_readfirstlane((int)threadIdx.x / S::LPA);
        const int rest = threadIdx.x % S::LPA;
        const int e = rest % EB, f = rest / EB;
        if (rest >= NF * EB || e >= ne) return;
        if (a == 0) {
            face_flux<DIM, P, 0, EB, SAVE>(m, ops, ph, s_u, s_t, s_qp, s_ih, e, f, k0 + e, Fs, Jp, sv);
        } else if (a == 1) {
            face_flux<DIM, P, 1, EB, SAVE>(m, ops, ph, s_u, s_t, s_qp, s_ih, e, f, k0 + e, Fs, Jp, sv);
        } else {
            if constexpr (DIM == 3) face_flux<DIM, P, 2, EB, SAVE>(m, ops, ph, s_u, s_t, s_qp, s_ih, e, f, k0 + e, Fs, Jp, sv);
        }
        return;
    } else {
        // wavefront pair per direction: 2a viscous, 2a + 1 Roe; one face point per lane
        const int w = __builtin_amdgcn_readfirstlane((int)threadIdx.x / S::LPA);
        const int a = w >> 1;
        const bool roe_wave = (w & 1) != 0;
        const int rest = threadIdx.x % S::LPA;
        const int e = rest % EB, f = rest / EB;
        const bool active = rest < NF * EB && e < ne;
        const int k = k0 + e;
        double Fr[NV];
        if (active) {
            if (!roe_wave) {
                auto visc = [&](auto Ac) {
                    constexpr int A = decltype(Ac)::value;
                    double qL[NV], qR[NV], g[DIM][NV], Sn[NV], Fv[NV];
                    plus_face_state<DIM, P, A, EB, EB>(ops, s_u, s_t, s_qp, s_ih, e, f, qL, qR, g, Sn);
#pragma unroll
                    for (int v = 0; v < NV; ++v) Jp[((size_t)(A * NV + v) * NF + f) * m.Ne + k] = qR[v] - qL[v];
                    if (SAVE) {
#pragma unroll
                        for (int v = 0; v < NV; ++v) {
                            const size_t o = ((size_t)(A * NV + v) * NF + f) * m.Ne + k;
                            sv.Qs[o] = qR[v];
                            sv.Qp[o] = qL[v];
                            sv.Sn[o] = Sn[v];
#pragma unroll
                            for (int c = 0; c < DIM; ++c) {
                                if (c == A) continue;
                                const int cc = c < A ? c : c - 1;
                                sv.Gt[((size_t)((A * (DIM - 1) + cc) * NV + v) * NF + f) * m.Ne + k] = g[c][v];
                            }
                        }
                    }
                    PState<DIM> sL;
                    pstate<DIM>(ph, qL, sL);
                    VGrad<DIM> vg;
                    vgrad<DIM>(sL, g, vg);
                    viscous_dir<DIM>(ph, A, sL, vg, Fv);
#pragma unroll
                    for (int v = 0; v < NV; ++v) s_x[((A * NV + v) * NF + f) * EB + e] = Fv[v] + ph.tau * (qR[v] - qL[v]);
                };
                if (a == 0) visc(std::integral_constant<int, 0>{});
                else if (a == 1) visc(std::integral_constant<int, 1>{});
                else if constexpr (DIM == 3) visc(std::integral_constant<int, 2>{});
            } else {
                double qL[NV], qR[NV];
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    const int fb = (a * NV + v) * NF + f;
                    qL[v] = s_qp[fb * EB + e];
                    qR[v] = s_t[fb * EB + e];
                }
                if (a == 0) roe<DIM>(ph, 0, qL, qR, Fr);
                else if (a == 1) roe<DIM>(ph, 1, qL, qR, Fr);
                else roe<DIM>(ph, DIM - 1, qL, qR, Fr);
            }
        }
        __syncthreads();
        if (!active || !roe_wave) return;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const int fb = (a * NV + v) * NF + f;
            Fs[(size_t)fb * m.Ne + k] = Fr[v] - s_x[fb * EB + e];
        }
    }
}

// Divergence part of R at solution point i of slot e (lane active), for EB
// slots staged as: s_u the state [v][i][slot] (overwritten by the fluxes,
// one direction at a time), s_t the state jumps q* - q+ on the + faces
// [a][v][f][slot], s_fm / s_fp the common fluxes on the - / + faces
// [a][v][f][slot] (overwritten by the flux jumps F* - f-/+), s_ih = 2/h with
// slot stride IHS.  Every lane of the workgroup calls it (it holds barriers);
// acc receives sum_a (2/h_a)[D f_a + (F*- - f-) gL' + (F*+ - f+) gR'] = -R.
template <int DIM, int P, int EB, int IHS>
__device__ __forceinline__ void divergence(const Ops1D &ops, const Phys &ph, double *s_u, const double *s_t,
                                           double *s_fm, double *s_fp, const double *s_ih, bool active, int e,
                                           int i, double (&acc)[DIM + 2]) {
    using S = Shape<DIM, P>;
    constexpr int NV = S::NV, NP = S::NP, NF = S::NF;
    PState<DIM> st;
    VGrad<DIM> vg;
    if (active) {
        double g[DIM][NV];
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            int f, ic;
            S::split(i, c, f, ic);
            const double ih = s_ih[sidx<IHS>(c, e)];
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                double d = 0.0;
#pragma unroll
                for (int j = 0; j < P; ++j) d += ops.D[ic][j] * s_u[(v * NP + S::line(c, f, j)) * EB + e];
                d += s_t[((c * NV + v) * NF + f) * EB + e] * ops.gRd[ic];
                g[c][v] = ih * d;
            }
        }
        double q[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) q[v] = s_u[(v * NP + i) * EB + e];
        pstate<DIM>(ph, q, st);
        vgrad<DIM>(st, g, vg);
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = 0.0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        double F[NV];
        if (active) {
            double FI[NV], FV[NV];
            inviscid_dev<DIM>(ph, a, st, FI);
            viscous_dir<DIM>(ph, a, st, vg, FV);
#pragma unroll
            for (int v = 0; v < NV; ++v) F[v] = FI[v] - FV[v];
        }
        __syncthreads();  // every read of s_u (state or previous flux) is done
        if (active) {
#pragma unroll
            for (int v = 0; v < NV; ++v) s_u[(v * NP + i) * EB + e] = F[v];
        }
        __syncthreads();
        // flux jumps on both faces normal to a
        for (int t2 = threadIdx.x; t2 < NV * NF * EB; t2 += blockDim.x) {
            const int e2 = t2 % EB;
            const int r = t2 / EB;
            const int f = r % NF, v = r / NF;
            double fm = 0.0, fp = 0.0;
#pragma unroll
            for (int j = 0; j < P; ++j) {
                const double xv = s_u[(v * NP + S::line(a, f, j)) * EB + e2];
                fm += ops.bm[j] * xv;
                fp += ops.bp[j] * xv;
            }
            const int fi = ((a * NV + v) * NF + f) * EB + e2;
            s_fm[fi] -= fm;
            s_fp[fi] -= fp;
        }
        __syncthreads();
        if (active) {
            int f, ia;
            S::split(i, a, f, ia);
            const double ih = s_ih[sidx<IHS>(a, e)];
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                double d = 0.0;
#pragma unroll
                for (int j = 0; j < P; ++j) d += ops.D[ia][j] * s_u[(v * NP + S::line(a, f, j)) * EB + e];
                const int fi = ((a * NV + v) * NF + f) * EB + e;
                d += s_fm[fi] * ops.gLd[ia] + s_fp[fi] * ops.gRd[ia];
                acc[v] += ih * d;
            }
        }
    }
}

struct OutK {
    double *r;
    const double *r0;
    const double *x;
    const double *vdir;
    double sigma;
    double dscale;
};

// Volume kernel.  In 2D every direction's flux is staged at once, so one
// evaluation takes five barriers (staging; state read; fluxes written; flux
// jumps formed; divergence terms exchanged) instead of three per direction,
// the flux jumps of all directions are formed in one pass, and two lanes
// serve each (point, slot), one per direction, each finishing half of the
// variables; the fluxes overlay the staged state and state jumps, which are
// dead by then (64x64 p = 4 linearised inside the stage: 11.3 -> 10.3 us,
// p = 2: 10.6 -> 8.2 us).  In 3D the staged fluxes would take 46 KB of LDS per workgroup,
// three workgroups per CU instead of four, and the kernel ran slower (207 ->
// 232 us at 32^3 p = 3): there it stages one direction at a time
// (divergence()).  Same arithmetic, in the same order, either way.
template <int DIM, int P, int MODE, int OUT>
__global__ void __launch_bounds__((Shape<DIM, P>::NTV))
k_volume(MeshK m, SrcK src, Ops1D ops_in, Phys ph, const double *__restrict__ Jp, const double *__restrict__ Fs,
         OutK o) {
    using S = Shape<DIM, P>;
    constexpr int EB = S::EB, NV = S::NV, NP = S::NP, NF = S::NF;
    constexpr int NFACE = DIM * NV * NF * EB;
    constexpr int NSTATE = NV * NP * EB;
    constexpr bool BATCH = (DIM == 2);
    constexpr int NA = (BATCH && DIM * NSTATE > NSTATE + NFACE) ? DIM * NSTATE : NSTATE + NFACE;
    __shared__ Ops1D ops;
    __shared__ double s_a[NA];      // the state [v][i][slot], the state jumps q* - q+ [a][v][f][slot]; then the fluxes [a][v][i][slot]
    __shared__ double s_fm[NFACE];  // F* on the - faces, then F* - f^-
    __shared__ double s_fp[NFACE];  // F* on the + faces, then F* - f^+
    __shared__ double s_ih[DIM * EB];
    __shared__ double s_x[BATCH ? NSTATE : 1];  // 2D: the divergence terms one half hands to the other
    double *s_u = s_a, *s_t = s_a + NSTATE;
    if (threadIdx.x == 0) ops = ops_in;
    const int k0 = xcd_block(blockIdx.x, gridDim.x) * EB;
    const int ne = min(EB, m.Ne - k0);
    const double alpha = (MODE == SRC_AXPY) ? sval(src.alpha) : 0.0;
    stage_state<DIM, P, MODE, EB, false>(m, src, ops_in, Jp, k0, ne, s_u, s_t, s_ih, alpha);
    for (int t = threadIdx.x; t < NFACE; t += blockDim.x) {
        const int e = t % EB;
        const int r = t / EB;  // (a * NV + v) * NF + f
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
    // 2D: two halves of NT lanes, half h taking direction h
    const int h = BATCH ? __builtin_amdgcn_readfirstlane((int)threadIdx.x / S::NT) : 0;
    const int t = BATCH ? (int)threadIdx.x - h * S::NT : (int)threadIdx.x;
    const int e = t % EB, i = t / EB;
    const bool active = (t < NP * EB) && (e < ne);
    double acc[NV];
    if constexpr (!BATCH) {
        divergence<DIM, P, EB, EB>(ops, ph, s_u, s_t, s_fm, s_fp, s_ih, active, e, i, acc);
        if (!active) return;
    } else {
        // two lanes per (point, slot): half h forms direction h's flux and
        // divergence; the halves meet through LDS, each finishing half of
        // the variables
        double F[NV];
        if (active) {
            double g[DIM][NV];
#pragma unroll
            for (int c = 0; c < DIM; ++c) {
                int f, ic;
                S::split(i, c, f, ic);
                const double ih = s_ih[c * EB + e];
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    double d = 0.0;
#pragma unroll
                    for (int j = 0; j < P; ++j) d += ops.D[ic][j] * s_u[(v * NP + S::line(c, f, j)) * EB + e];
                    d += s_t[((c * NV + v) * NF + f) * EB + e] * ops.gRd[ic];
                    g[c][v] = ih * d;
                }
            }
            double q[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) q[v] = s_u[(v * NP + i) * EB + e];
            PState<DIM> st;
            VGrad<DIM> vg;
            pstate<DIM>(ph, q, st);
            vgrad<DIM>(st, g, vg);
            auto flux = [&](auto Ac) {
                constexpr int A = decltype(Ac)::value;
                double FI[NV], FV[NV];
                inviscid_dev<DIM>(ph, A, st, FI);
                viscous_dir<DIM>(ph, A, st, vg, FV);
#pragma unroll
                for (int v = 0; v < NV; ++v) F[v] = FI[v] - FV[v];
            };
            if (h == 0) flux(std::integral_constant<int, 0>{});
            else flux(std::integral_constant<int, 1>{});
        }
        __syncthreads();  // every read of the state and the jumps is done
        if (active) {
#pragma unroll
            for (int v = 0; v < NV; ++v) s_a[((h * NV + v) * NP + i) * EB + e] = F[v];
        }
        __syncthreads();
        // flux jumps on both faces normal to every axis
        for (int t2 = threadIdx.x; t2 < NFACE; t2 += blockDim.x) {
            const int e2 = t2 % EB;
            int r = t2 / EB;
            const int f = r % NF;
            r /= NF;
            const int v = r % NV, a = r / NV;
            const double *x = s_a + (a * NV + v) * NP * EB + e2;
            double fm = 0.0, fp = 0.0;
#pragma unroll
            for (int j = 0; j < P; ++j) {
                const double xv = x[S::line(a, f, j) * EB];
                fm += ops.bm[j] * xv;
                fp += ops.bp[j] * xv;
            }
            s_fm[t2] -= fm;
            s_fp[t2] -= fp;
        }
        __syncthreads();
        // direction h's divergence term d (before the 2/h factor), for every variable
        double dd[NV];
        if (active) {
            int f, ia;
            S::split(i, h, f, ia);
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                double d = 0.0;
#pragma unroll
                for (int j = 0; j < P; ++j) d += ops.D[ia][j] * s_a[((h * NV + v) * NP + S::line(h, f, j)) * EB + e];
                const int fi = ((h * NV + v) * NF + f) * EB + e;
                d += s_fm[fi] * ops.gLd[ia] + s_fp[fi] * ops.gRd[ia];
                dd[v] = d;
            }
#pragma unroll
            for (int v = 0; v < NV; ++v)
                if ((v < NV / 2) != (h == 0)) s_x[(v * NP + i) * EB + e] = dd[v];  // the other half finishes v
        }
        __syncthreads();
        if (!active) return;
        const double ih0 = s_ih[e], ih1 = s_ih[EB + e];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            acc[v] = 0.0;
            if ((v < NV / 2) == (h == 0)) {
                const double o = s_x[(v * NP + i) * EB + e];
                const double d0 = (h == 0) ? dd[v] : o, d1 = (h == 0) ? o : dd[v];
                acc[v] += ih0 * d0;
                acc[v] += ih1 * d1;
            }
        }
    }
    const int k = k0 + e;
    // the optional subtrahend x is tested once, outside the unrolled loop (a
    // test per variable inside it more than doubled the registers)
    const double *xs = o.x;
    // the variables this lane finishes (all of them but in the 2D two-lane form)
    auto mine = [&](int v) { return !BATCH || ((v < NV / 2) == (h == 0)); };
    if (OUT == OUT_R) {
#pragma unroll
        for (int v = 0; v < NV; ++v)
            if (mine(v)) o.r[((size_t)v * NP + i) * m.Ne + k] = -acc[v];
    } else if (xs) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            if (!mine(v)) continue;
            const size_t idx = ((size_t)v * NP + i) * m.Ne + k;
            o.r[idx] = o.sigma * o.vdir[idx] - (-acc[v] - o.r0[idx]) / (alpha * o.dscale) - xs[idx];
        }
    } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            if (!mine(v)) continue;
            const size_t idx = ((size_t)v * NP + i) * m.Ne + k;
            o.r[idx] = o.sigma * o.vdir[idx] - (-acc[v] - o.r0[idx]) / (alpha * o.dscale);
        }
    }
}

// ---------------------------------------------------------------------------
// element-Jacobi blocks by element-local one-sided differences
// ---------------------------------------------------------------------------
//
// Column j of B_k = sigma I - dR_k/dq_k is sigma e_j - (R_k(q + h e_j) - R_k(q)) / h
// with only element k perturbed.  R_k depends on the states of k and of its
// face neighbours; with k alone perturbed, the neighbours enter only through
// face data of the unperturbed state: the + neighbours' minus traces (q* on
// k's + faces) and, for each - face of k (owned by the - neighbour m), m's
// + trace, the D part of m's normal gradient and m's tangential gradient
// components there -- the normal gradient at that face changes with k
// through q* only.  These are saved by one base evaluation; each workgroup
// then evaluates R_k for EB columns of one element (the slots) at a time,
// with the same arithmetic as a global evaluation.  A workgroup takes
// `groups` such column groups of one element in turn: the element's state
// and its neighbours' face data are read once (scattered reads, one cache
// line per value in the element-fastest layout) and kept in LDS for all of
// them.

// column groups per workgroup: 32^3 p = 3, 320-column blocks: 64.6 ms with
// one group per workgroup, 55.3 ms with 4, 52.7 with 16, 52.2 with 80
constexpr int kFormGroups = 16;

struct FormK {
    const double *dq;  // linearisation point
    FaceSave sv;       // base face data
    const double *r0;  // R at the linearisation point
    double *blocks;    // [Ne][nb][nb], column-major per block
    double sigma;
    int nb;
    int groups;        // column groups of EB per workgroup
};

template <int DIM, int P>
__global__ void __launch_bounds__((Shape<DIM, P>::NT)) k_ej_form(MeshK m, Ops1D ops_in, Phys ph, FormK fk) {
    using S = Shape<DIM, P>;
    constexpr int EB = S::EB, NV = S::NV, NP = S::NP, NF = S::NF;
    constexpr int NFACE = DIM * NV * NF * EB;
    constexpr int NSH = DIM * NV * NF;
    // a copy of the element's state at the linearisation point, except for
    // the 3D p = 2 blocks (135 columns), where it would leave LDS for two
    // workgroups per CU instead of three: those read the state from memory
    constexpr bool KEEPQ = !(DIM == 3 && P == 3);
    __shared__ Ops1D ops;
    __shared__ double s_q0[KEEPQ ? NV * NP : 1];
    __shared__ double s_u[NV * NP * EB];   // perturbed states, then the flux of one direction
    __shared__ double s_qp[NFACE];         // own + traces, then the jumps q* - q+
    __shared__ double s_qm[NFACE];         // own - traces (q* on the - faces)
    __shared__ double s_fm[NFACE];         // F* on the - faces, then F* - f^-
    __shared__ double s_fp[NFACE];         // F* on the + faces, then F* - f^+
    __shared__ double s_tn[NSH];           // q* on the + faces
    __shared__ double s_mq[NSH];           // - neighbours' + traces
    __shared__ double s_ms[NSH];           // - neighbours' normal-gradient D parts
    __shared__ double s_mg[DIM > 1 ? (DIM - 1) * NSH : 1];  // - neighbours' tangential gradients
    __shared__ double s_ih[DIM], s_ihm[DIM];
    if (threadIdx.x == 0) ops = ops_in;
    const int nb = fk.nb;
    const int ncb = (nb + EB - 1) / EB;
    const int nwe = (ncb + fk.groups - 1) / fk.groups;  // workgroups per element
    const int b = xcd_block(blockIdx.x, gridDim.x);
    const int k = b / nwe;
    const int g0 = (b % nwe) * fk.groups, g1 = min(ncb, g0 + fk.groups);
    if constexpr (KEEPQ)
        for (int t = threadIdx.x; t < NV * NP; t += blockDim.x) s_q0[t] = fk.dq[(size_t)t * m.Ne + k];
    for (int t = threadIdx.x; t < NSH; t += blockDim.x) {
        const int a = t / (NV * NF);
        const int mm = neighbour(m, k, a, -1);
        s_tn[t] = fk.sv.Qs[(size_t)t * m.Ne + k];
        s_mq[t] = fk.sv.Qp[(size_t)t * m.Ne + mm];
        s_ms[t] = fk.sv.Sn[(size_t)t * m.Ne + mm];
    }
    for (int t = threadIdx.x; t < (DIM - 1) * NSH; t += blockDim.x) {
        const int a = t / ((DIM - 1) * NV * NF);
        s_mg[t] = fk.sv.Gt[(size_t)t * m.Ne + neighbour(m, k, a, -1)];
    }
    if (threadIdx.x < DIM) {
        const int a = threadIdx.x;
        int c[3];
        coords(m, k, c);
        s_ih[a] = m.inv2h[a][c[a]];
        s_ihm[a] = m.inv2h[a][c[a] > 0 ? c[a] - 1 : m.n[a] - 1];
    }
    for (int g = g0; g < g1; ++g) {
        const int col0 = g * EB;
        const int ncol = min(EB, nb - col0);
        // the lane index, re-read each group: the index arithmetic of the
        // loops below is then not hoisted out of this loop, where it would
        // hold registers for the whole kernel (200 instead of 144 VGPRs)
        int tid;
        __asm__ volatile("v_mov_b32 %0, %1" : "=v"(tid) : "v"((int)threadIdx.x));
        __syncthreads();  // s_q0 staged; the previous group's reads of s_u are done
        for (int t = tid; t < NV * NP * EB; t += blockDim.x) {
            const int e = t % EB, vi = t / EB;
            const int v = vi / NP;
            double u = KEEPQ ? s_q0[vi] : fk.dq[(size_t)vi * m.Ne + k];
            if (e < ncol && vi == col0 + e) u = u + fd_step(ph.qinf[v], u);
            s_u[t] = u;
        }
        __syncthreads();
        // own traces of every slot
        for (int t = tid; t < NFACE; t += blockDim.x) {
            const int e = t % EB;
            int r = t / EB;
            const int f = r % NF;
            r /= NF;
            const int v = r % NV, a = r / NV;
            double sp = 0.0, sm = 0.0;
#pragma unroll
            for (int j = 0; j < P; ++j) {
                const double x = s_u[(v * NP + S::line(a, f, j)) * EB + e];
                sp += ops.bp[j] * x;
                sm += ops.bm[j] * x;
            }
            s_qp[t] = sp;
            s_qm[t] = sm;
        }
        __syncthreads();
        // common fluxes on the 2 DIM faces of every slot
        for (int t = tid; t < 2 * DIM * NF * EB; t += blockDim.x) {
            const int e = t % EB;
            int r = t / EB;
            const int f = r % NF;
            r /= NF;
            const int a = r % DIM, side = r / DIM;
            double qL[NV], qR[NV], g2[DIM][NV], F[NV];
            auto minus_face = [&](auto Ac) {
                constexpr int A = decltype(Ac)::value;
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    const int fb = (A * NV + v) * NF + f;
                    qL[v] = s_mq[fb];
                    qR[v] = s_qm[fb * EB + e];
                    double d = s_ms[fb];
                    d += (qR[v] - qL[v]) * ops.cgp;
                    g2[A][v] = s_ihm[A] * d;
#pragma unroll
                    for (int c = 0; c < DIM; ++c) {
                        if (c == A) continue;
                        const int cc = c < A ? c : c - 1;
                        g2[c][v] = s_mg[((A * (DIM - 1) + cc) * NV + v) * NF + f];
                    }
                }
                common_flux<DIM, A>(ph, qL, qR, g2, F);
#pragma unroll
                for (int v = 0; v < NV; ++v) s_fm[((A * NV + v) * NF + f) * EB + e] = F[v];
            };
            auto plus_face = [&](auto Ac) {
                constexpr int A = decltype(Ac)::value;
                double Sn[NV];
                plus_face_state<DIM, P, A, EB, 0>(ops, s_u, s_tn, s_qp, s_ih, e, f, qL, qR, g2, Sn);
                common_flux<DIM, A>(ph, qL, qR, g2, F);
#pragma unroll
                for (int v = 0; v < NV; ++v) s_fp[((A * NV + v) * NF + f) * EB + e] = F[v];
            };
            using A0 = std::integral_constant<int, 0>;
            using A1 = std::integral_constant<int, 1>;
            using A2 = std::integral_constant<int, (DIM == 3 ? 2 : 1)>;
            if (side == 0) {
                if (a == 0) plus_face(A0{});
                else if (a == 1) plus_face(A1{});
                else if constexpr (DIM == 3) plus_face(A2{});
            } else {
                if (a == 0) minus_face(A0{});
                else if (a == 1) minus_face(A1{});
                else if constexpr (DIM == 3) minus_face(A2{});
            }
        }
        __syncthreads();
        // state jumps q* - q+ on the + faces
        for (int t = tid; t < NFACE; t += blockDim.x) s_qp[t] = s_tn[t / EB] - s_qp[t];
        __syncthreads();
        const int t = tid;
        const int e = t % EB, i = t / EB;
        const bool active = (t < NP * EB);
        double acc[NV];
        divergence<DIM, P, EB, 0>(ops, ph, s_u, s_qp, s_fm, s_fp, s_ih, active, e, i, acc);
        if (active && e < ncol) {
            const int col = col0 + e;
            const double base = KEEPQ ? s_q0[col] : fk.dq[(size_t)col * m.Ne + k];
            const double hact = (base + fd_step(ph.qinf[col / NP], base)) - base;
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const double R = -acc[v];
                const int row = v * NP + i;
                double val = -(R - fk.r0[(size_t)row * m.Ne + k]) / hact;
                if (row == col) val += fk.sigma;
                fk.blocks[(size_t)k * nb * nb + (size_t)col * nb + row] = val;
            }
        }
    }
}

// One evaluation on mesh m with face buffers Jp, Fs ([dim][nv][NF][m.Ne]).
template <int DIM, int P, int MODE, int OUT>
hipError_t run_on(const frpmg_ctx *ctx, const Level &L, const MeshK &m, double *Jp, double *Fs,
                  const ResidualArgs &a, const FaceSave *save, hipStream_t s) {
    using S = Shape<DIM, P>;
    SrcK src{a.dq, a.v, a.alpha, S::NP};
    const dim3 g1((m.Ne + S::EBF - 1) / S::EBF);
    if (save) {
        hipLaunchKernelGGL((k_faces<DIM, P, MODE, true>), g1, dim3(S::NTF2), 0, s, m, src, L.ops, ctx->phys, Jp, Fs,
                           *save);
    } else {
        hipLaunchKernelGGL((k_faces<DIM, P, MODE, false>), g1, dim3(S::NTF2), 0, s, m, src, L.ops, ctx->phys, Jp,
                           Fs, FaceSave{nullptr, nullptr, nullptr, nullptr});
    }
    OutK o{a.r, a.r0, a.x, a.v, a.sigma, a.dscale};
    hipLaunchKernelGGL((k_volume<DIM, P, MODE, OUT>), dim3((m.Ne + S::EB - 1) / S::EB), dim3(S::NTV), 0, s, m, src,
                       L.ops, ctx->phys, Jp, Fs, o);
    return hipGetLastError();
}

template <int DIM, int P, int MODE, int OUT>
hipError_t run(const frpmg_ctx *ctx, const Level &L, const ResidualArgs &a, const FaceSave *save, hipStream_t s) {
    return run_on<DIM, P, MODE, OUT>(ctx, L, ctx->mesh, L.Jp, L.Fs, a, save, s);
}

template <int DIM, int P>
hipError_t dispatch_modes(const frpmg_ctx *ctx, const Level &L, const ResidualArgs &a, const FaceSave *save,
                          hipStream_t s) {
    if (a.src == SRC_PLAIN && a.out == OUT_R) return run<DIM, P, SRC_PLAIN, OUT_R>(ctx, L, a, save, s);
    if (save) return hipErrorInvalidValue;
    if (a.src == SRC_AXPY && a.out == OUT_R) return run<DIM, P, SRC_AXPY, OUT_R>(ctx, L, a, nullptr, s);
    if (a.src == SRC_AXPY && a.out == OUT_LIN) return run<DIM, P, SRC_AXPY, OUT_LIN>(ctx, L, a, nullptr, s);
    return hipErrorInvalidValue;
}

template <int DIM, int P>
hipError_t form(const frpmg_ctx *ctx, const Level &L, const double *dq, double sigma, double *out, hipStream_t s) {
    using S = Shape<DIM, P>;
    const MeshK &m = ctx->mesh;
    const FaceSave sv{L.fQs, L.fQp, L.fSn, L.fGt};
    ResidualArgs a;
    a.src = SRC_PLAIN;
    a.dq = dq;
    a.out = OUT_R;
    a.r = L.r0;
    hipError_t err = run<DIM, P, SRC_PLAIN, OUT_R>(ctx, L, a, &sv, s);
    if (err != hipSuccess) return err;
    const int ncb = (L.nb + S::EB - 1) / S::EB;
    const int groups = kFormGroups;
    const size_t nblk = (size_t)m.Ne * ((ncb + groups - 1) / groups);
    if (nblk > 0x7fffffff) return hipErrorInvalidValue;
    FormK fk{dq, sv, L.r0, out, sigma, L.nb, groups};
    hipLaunchKernelGGL((k_ej_form<DIM, P>), dim3((unsigned)nblk), dim3(S::NT), 0, s, m, L.ops, ctx->phys, fk);
    return hipGetLastError();
}


// ---------------------------------------------------------------------------
// mixed polynomial degrees (p-adaptation, Sec. 3.3)
// ---------------------------------------------------------------------------
//
// Element k has P_k points per direction; states are padded to the level's
// largest P (point stride NpM) and face arrays to its NFM points per face.
// The elements of each point count form a class, launched with that count as
// a compile-time constant (element ids from a list, so every wavefront runs
// one degree).  A face between elements of equal degree is treated exactly as
// in the uniform kernels.  At a face between different degrees, the common
// solution seen from the -axis element is the L2 projection of the +axis
// element's trace onto its face points (exact interpolation when the -axis
// side has the larger degree); the common flux is formed at the points of the
// larger degree (the mortar) from both traces and the -axis element's
// gradient trace projected there, and is returned to both sides by L2
// projection, which keeps its integral over the face (k_pa_mortar).

constexpr int kMaxNF3 = 16;  // face points of a 3D element (p <= 3)

struct PaK {
    const int *Pk;         // points per direction of every element
    const int *list;       // element ids of the launched class
    int count;             // elements in the list
    int ne0;               // elements per mesh copy: id k is element k % ne0 of copy k / ne0
    int NpM, NFM;          // padded points per element / per face
    const PaTables *tab;   // operators of every degree
    double *Fm;            // common flux on - faces [dim][nv][NFM][Ne]
    double *Mq, *Mn, *Mg;  // mortar inputs, on the + face of the -axis element
};

// + neighbour of element id k along a, within k's mesh copy
__device__ __forceinline__ int pa_plus_neighbour(const MeshK &m, const PaK &pk, int k, int a) {
    const int kb = (k / pk.ne0) * pk.ne0;
    return kb + neighbour(m, k - kb, a, +1);
}

__device__ __forceinline__ double pa_inv2h(const MeshK &m, const PaK &pk, int k, int a) {
    int c[3];
    coords(m, k % pk.ne0, c);
    return m.inv2h[a][c[a]];
}

// local point on the line along axis a through face point f, position j (P at run time)
__device__ __forceinline__ int line_rt(int dim, int P, int a, int f, int j) {
    if (a == 0) return j + P * f;
    if (dim == 2) return f + P * j;
    if (a == 1) return (f % P) + P * (j + P * (f / P));
    return f + P * P * j;
}

// value at face point fb (Pb points per direction) of the L2 projection of the
// face function x (Pa points per direction, entry fa at x[fa * xs]): the tensor
// product of the 1D projections over the face's dim - 1 directions
__device__ __forceinline__ double face_map_pt(const PaTables *tab, int dim, int Pa, int Pb, int fb,
                                              const double *x, size_t xs) {
    const int b0 = fb % Pb, b1 = fb / Pb;
    const int nfa = (dim == 2) ? Pa : Pa * Pa;
    double s = 0.0;
    for (int fa = 0; fa < nfa; ++fa) {
        const int a0 = fa % Pa, a1 = fa / Pa;
        double c = tab->proj[Pa][Pb][b0][a0];
        if (dim == 3) c *= tab->proj[Pa][Pb][b1][a1];
        s += c * x[(size_t)fa * xs];
    }
    return s;
}

// One + face point of a class-P element: the state jump and, at a face of
// equal degrees, the common flux (written for both elements); at a face of
// different degrees, the mortar inputs.
template <int DIM, int P, int A, int EB>
__device__ __forceinline__ void pa_face_flux(const MeshK &m, const Ops1D &ops, const Phys &ph, const PaK &pk,
                                             const double *s_u, const double *s_t, const double *s_qp,
                                             const double *s_ih, int e, int f, int k, int kn, int pn,
                                             double *__restrict__ Fs, double *__restrict__ Jp) {
    constexpr int NV = DIM + 2;
    double qL[NV], qR[NV], g[DIM][NV], Sn[NV], F[NV];
    plus_face_state<DIM, P, A, EB, EB>(ops, s_u, s_t, s_qp, s_ih, e, f, qL, qR, g, Sn);
    const size_t Ne = (size_t)m.Ne;
#pragma unroll
    for (int v = 0; v < NV; ++v) Jp[((size_t)(A * NV + v) * pk.NFM + f) * Ne + k] = qR[v] - qL[v];
    if (pn == P) {
        common_flux<DIM, A>(ph, qL, qR, g, F);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const size_t o = ((size_t)(A * NV + v) * pk.NFM + f) * Ne;
            Fs[o + k] = F[v];
            pk.Fm[o + kn] = F[v];
        }
    } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            pk.Mq[((size_t)(A * NV + v) * pk.NFM + f) * Ne + k] = qL[v];
#pragma unroll
            for (int c = 0; c < DIM; ++c)
                pk.Mg[(((size_t)(A * DIM + c) * NV + v) * pk.NFM + f) * Ne + k] = g[c][v];
        }
    }
}

// LDS of one class's face workgroup, in doubles: the class's 1D operators,
// the state [v][i][slot], the + neighbours' minus traces at their own points
// [a][v][f][slot], q* and the own + traces on the + faces at own points,
// 2/h, then the slots' element ids and their + neighbours' ids and point counts.
template <int DIM, int P>
struct PaFacesLds {
    using S = Shape<DIM, P>;
    static constexpr int EB = S::EBF, NV = S::NV, NP = S::NP, NF = S::NF;
    static constexpr int NFN = (DIM == 2) ? kMaxP : kMaxNF3;  // a neighbour's face points, at most
    static constexpr int NFACE = DIM * NV * NF * EB;
    static constexpr int OPS = (int)(sizeof(Ops1D) / sizeof(double));
    static constexpr int U = OPS, TN = U + NV * NP * EB, T = TN + DIM * NV * NFN * EB, QP = T + NFACE,
                         IH = QP + NFACE, INTS = IH + DIM * EB;
    static constexpr int DOUBLES = INTS + (EB + 2 * DIM * EB + 1) / 2;
};

// + faces of the class-P elements of workgroup blk of the class (one lane
// per face point, as k_faces).
template <int DIM, int P, int MODE>
__device__ __forceinline__ void pa_faces_body(const MeshK &m, const SrcK &src, const Phys &ph, const PaK &pk,
                                              double *__restrict__ Jp, double *__restrict__ Fs, int blk,
                                              double *lds) {
    using S = Shape<DIM, P>;
    using LD = PaFacesLds<DIM, P>;
    constexpr int EB = S::EBF, NV = S::NV, NP = S::NP, NF = S::NF;
    constexpr int NFACE = DIM * NV * NF * EB;
    constexpr int NFN = LD::NFN;
    const Ops1D &ops = *reinterpret_cast<const Ops1D *>(lds);
    double *s_u = lds + LD::U;
    double *s_tn = lds + LD::TN;
    double *s_t = lds + LD::T;
    double *s_qp = lds + LD::QP;
    double *s_ih = lds + LD::IH;
    int *s_k = reinterpret_cast<int *>(lds + LD::INTS);
    int *s_kn = s_k + EB, *s_pn = s_kn + DIM * EB;
    {
        const double *src_ops = reinterpret_cast<const double *>(&pk.tab->ops[P]);
        for (int t = threadIdx.x; t < LD::OPS; t += blockDim.x) lds[t] = src_ops[t];
    }
    const int b0 = blk * EB;
    const int ne = min(EB, pk.count - b0);
    const double alpha = (MODE == SRC_AXPY) ? sval(src.alpha) : 0.0;
    for (int t = threadIdx.x; t < EB; t += blockDim.x) s_k[t] = (t < ne) ? pk.list[b0 + t] : 0;
    __syncthreads();
    for (int t = threadIdx.x; t < DIM * EB; t += blockDim.x) {
        const int e = t % EB, a = t / EB;
        int kn = 0, pn = P;
        double ih = 0.0;
        if (e < ne) {
            const int k = s_k[e];
            kn = pa_plus_neighbour(m, pk, k, a);
            pn = pk.Pk[kn];
            ih = pa_inv2h(m, pk, k, a);
        }
        s_kn[t] = kn;
        s_pn[t] = pn;
        s_ih[t] = ih;
    }
    for (int t = threadIdx.x; t < NV * NP * EB; t += blockDim.x) {
        const int e = t % EB, vi = t / EB;
        s_u[t] = (e < ne) ? load_state<MODE>(src, m, vi / NP, vi % NP, s_k[e], alpha) : 0.0;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < DIM * NV * NFN * EB; t += blockDim.x) {
        const int e = t % EB;
        int r = t / EB;
        const int f = r % NFN;
        r /= NFN;
        const int v = r % NV, a = r / NV;
        const int pn = s_pn[a * EB + e];
        double val = 0.0;
        if (e < ne && f < ((DIM == 2) ? pn : pn * pn)) {
            const int kn = s_kn[a * EB + e];
            if (pn == P) {
#pragma unroll
                for (int j = 0; j < P; ++j) val += ops.bm[j] * load_state<MODE>(src, m, v, S::line(a, f, j), kn, alpha);
            } else {
                const double *bmn = pk.tab->ops[pn].bm;
                for (int j = 0; j < pn; ++j)
                    val += bmn[j] * load_state<MODE>(src, m, v, line_rt(DIM, pn, a, f, j), kn, alpha);
            }
        }
        s_tn[t] = val;
    }
    for (int t = threadIdx.x; t < NFACE; t += blockDim.x) {
        const int e = t % EB;
        int r = t / EB;
        const int f = r % NF;
        r /= NF;
        const int v = r % NV, a = r / NV;
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < P; ++j) s += ops.bp[j] * s_u[(v * NP + S::line(a, f, j)) * EB + e];
        s_qp[t] = s;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < NFACE; t += blockDim.x) {
        const int e = t % EB;
        int r = t / EB;
        const int f = r % NF;
        r /= NF;
        const int v = r % NV, a = r / NV;
        const int pn = s_pn[a * EB + e];
        const double *tn = &s_tn[(a * NV + v) * NFN * EB + e];
        s_t[t] = (pn == P) ? tn[f * EB] : face_map_pt(pk.tab, DIM, pn, P, f, tn, EB);
    }
    // mixed faces: the neighbour's trace at its own points, for the mortar
    for (int t = threadIdx.x; t < DIM * NV * NFN * EB; t += blockDim.x) {
        const int e = t % EB;
        int r = t / EB;
        const int f = r % NFN;
        r /= NFN;
        const int v = r % NV, a = r / NV;
        const int pn = s_pn[a * EB + e];
        if (e < ne && pn != P && f < ((DIM == 2) ? pn : pn * pn))
            pk.Mn[((size_t)(a * NV + v) * pk.NFM + f) * m.Ne + s_k[e]] = s_tn[t];
    }
    __syncthreads();
    const int a = __builtin_amdgcn_readfirstlane((int)threadIdx.x / S::LPA);
    const int rest = threadIdx.x % S::LPA;
    const int e = rest % EB, f = rest / EB;
    if (rest >= NF * EB || e >= ne) return;
    const int k = s_k[e], kn = s_kn[a * EB + e], pn = s_pn[a * EB + e];
    if (a == 0) {
        pa_face_flux<DIM, P, 0, EB>(m, ops, ph, pk, s_u, s_t, s_qp, s_ih, e, f, k, kn, pn, Fs, Jp);
    } else if (a == 1) {
        pa_face_flux<DIM, P, 1, EB>(m, ops, ph, pk, s_u, s_t, s_qp, s_ih, e, f, k, kn, pn, Fs, Jp);
    } else {
        if constexpr (DIM == 3) pa_face_flux<DIM, P, 2, EB>(m, ops, ph, pk, s_u, s_t, s_qp, s_ih, e, f, k, kn, pn, Fs, Jp);
    }
}

// face_map_pt with the 1D projection T (rows of kMaxP, T[b kMaxP + a]) and
// the input (contiguous) in LDS
__device__ __forceinline__ double face_map_lds(const double *T, int dim, int Pa, int Pb, int fb, const double *x) {
    const int b0 = fb % Pb, b1 = fb / Pb;
    const int nfa = (dim == 2) ? Pa : Pa * Pa;
    double s = 0.0;
    for (int fa = 0; fa < nfa; ++fa) {
        const int a0 = fa % Pa, a1 = fa / Pa;
        double c = T[b0 * kMaxP + a0];
        if (dim == 3) c *= T[b1 * kMaxP + a1];
        s += c * x[fa];
    }
    return s;
}

// The common flux on faces between elements of different degree.  The
// workgroup first stages the 1D projections and, for each of its faces, the
// mortar inputs (the -axis element's + trace and gradient trace, the +axis
// element's - trace) in LDS, all loads in flight at once; then one lane per
// mortar point forms the flux from the inputs projected there, and the
// lanes project it back onto the -axis element's + face (Fs) and the +axis
// element's - face (Fm).
template <int DIM>
__global__ void __launch_bounds__(64) k_pa_mortar(MeshK m, Phys ph, PaK pk, const int *__restrict__ faces,
                                                  int nfaces, double *__restrict__ Fs) {
    constexpr int NV = DIM + 2;
    constexpr int NFMM = (DIM == 2) ? kMaxP : kMaxNF3;
    constexpr int FB = 64 / NFMM;
    constexpr int NIN = (2 + DIM) * NV;  // q+ of the -axis element, q- of the +axis one, the gradient trace
    constexpr int NT = (kMaxP + 1) * (kMaxP + 1) * kMaxP * kMaxP;
    __shared__ double sT[NT];
    __shared__ double sIn[FB][NIN][NFMM];
    __shared__ double sF[FB][NV][NFMM];
    __shared__ int sk[FB], skn[FB], sa[FB], spk[FB], spn[FB];
    const int tid = threadIdx.x;
    const size_t Ne = (size_t)m.Ne;
    if (tid < FB) {
        const int fi = blockIdx.x * FB + tid;
        int k = 0, a = 0, kn = 0, Pk = 1, Pn = 1;
        if (fi < nfaces) {
            const int code = faces[fi];
            k = code >> 2;
            a = code & 3;
            kn = pa_plus_neighbour(m, pk, k, a);
            Pk = pk.Pk[k];
            Pn = pk.Pk[kn];
        }
        sk[tid] = k;
        skn[tid] = kn;
        sa[tid] = a;
        spk[tid] = (fi < nfaces) ? Pk : 0;
        spn[tid] = Pn;
    }
    {
        const double *tab = &pk.tab->proj[0][0][0][0];
        for (int t = tid; t < NT; t += 64) sT[t] = tab[t];
    }
    __syncthreads();
    for (int t = tid; t < FB * NIN * NFMM; t += 64) {
        const int slot = t / (NIN * NFMM), r = t % (NIN * NFMM);
        const int q = r / NFMM, f = r % NFMM;
        const int Pk = spk[slot];
        double val = 0.0;
        if (Pk > 0) {
            const int a = sa[slot], Pn = spn[slot];
            const int nfk = (DIM == 2) ? Pk : Pk * Pk, nfn = (DIM == 2) ? Pn : Pn * Pn;
            if (q < NV) {
                if (f < nfk) val = pk.Mq[((size_t)(a * NV + q) * pk.NFM + f) * Ne + sk[slot]];
            } else if (q < 2 * NV) {
                if (f < nfn) val = pk.Mn[((size_t)(a * NV + q - NV) * pk.NFM + f) * Ne + sk[slot]];
            } else {
                const int cv = q - 2 * NV;  // c * NV + v
                if (f < nfk) val = pk.Mg[((size_t)(a * DIM * NV + cv) * pk.NFM + f) * Ne + sk[slot]];
            }
        }
        sIn[slot][q][f] = val;
    }
    __syncthreads();
    const int slot = tid / NFMM, fm = tid % NFMM;
    const bool act = slot < FB && spk[slot < FB ? slot : 0] > 0;
    int a = 0, Pk = 1, Pn = 1, Pm = 1;
    if (act) {
        a = sa[slot];
        Pk = spk[slot];
        Pn = spn[slot];
        Pm = max(Pk, Pn);
    }
    if (act && fm < ((DIM == 2) ? Pm : Pm * Pm)) {
        const double *TkM = &sT[((Pk * (kMaxP + 1) + Pm) * kMaxP) * kMaxP];
        const double *TnM = &sT[((Pn * (kMaxP + 1) + Pm) * kMaxP) * kMaxP];
        double qL[NV], qR[NV], g[DIM][NV], F[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            qL[v] = (Pk == Pm) ? sIn[slot][v][fm] : face_map_lds(TkM, DIM, Pk, Pm, fm, sIn[slot][v]);
            qR[v] = (Pn == Pm) ? sIn[slot][NV + v][fm] : face_map_lds(TnM, DIM, Pn, Pm, fm, sIn[slot][NV + v]);
#pragma unroll
            for (int c = 0; c < DIM; ++c) {
                const double *x = sIn[slot][2 * NV + c * NV + v];
                g[c][v] = (Pk == Pm) ? x[fm] : face_map_lds(TkM, DIM, Pk, Pm, fm, x);
            }
        }
        if (a == 0) {
            common_flux<DIM, 0>(ph, qL, qR, g, F);
        } else if (a == 1) {
            common_flux<DIM, 1>(ph, qL, qR, g, F);
        } else {
            if constexpr (DIM == 3) common_flux<DIM, 2>(ph, qL, qR, g, F);
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) sF[slot][v][fm] = F[v];
    }
    __syncthreads();
    if (!act) return;
    const int k = sk[slot], kn = skn[slot];
    const int nfk = (DIM == 2) ? Pk : Pk * Pk, nfn = (DIM == 2) ? Pn : Pn * Pn;
    const double *TMk = &sT[((Pm * (kMaxP + 1) + Pk) * kMaxP) * kMaxP];
    const double *TMn = &sT[((Pm * (kMaxP + 1) + Pn) * kMaxP) * kMaxP];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const size_t o = ((size_t)(a * NV + v) * pk.NFM + fm) * Ne;
        if (fm < nfk) Fs[o + k] = (Pk == Pm) ? sF[slot][v][fm] : face_map_lds(TMk, DIM, Pm, Pk, fm, sF[slot][v]);
        if (fm < nfn) pk.Fm[o + kn] = (Pn == Pm) ? sF[slot][v][fm] : face_map_lds(TMn, DIM, Pm, Pn, fm, sF[slot][v]);
    }
}

// LDS of one class's volume workgroup (doubles): operators, state, state
// jumps and common fluxes on both face sets, 2/h, element ids.  One point per
// element (p = 0) takes 128 elements per 256-lane workgroup in 2D.
template <int DIM, int P>
struct PaVolLds {
    using S = Shape<DIM, P>;
    static constexpr int EB = (P == 1) ? (DIM == 2 ? 128 : 64) : S::EB;
    static constexpr int NV = S::NV, NP = S::NP, NF = S::NF;
    static constexpr int NFACE = DIM * NV * NF * EB;
    static constexpr int OPS = (int)(sizeof(Ops1D) / sizeof(double));
    static constexpr int U = OPS, T = U + NV * NP * EB, FM = T + NFACE, FP = FM + NFACE, IH = FP + NFACE,
                         INTS = IH + DIM * EB;
    static constexpr int DOUBLES = INTS + (EB + 1) / 2;
};

// Divergence of the class-P elements of workgroup blk of the class
// (k_volume with element ids from the list, padded strides and the - face
// fluxes from Fm); also writes the padding entries of the output (0).
template <int DIM, int P, int MODE, int OUT>
__device__ __forceinline__ void pa_volume_body(const MeshK &m, const SrcK &src, const Phys &ph, const PaK &pk,
                                               const double *__restrict__ Jp, const double *__restrict__ Fs,
                                               const OutK &o, int blk, double *lds) {
    using S = Shape<DIM, P>;
    using LD = PaVolLds<DIM, P>;
    constexpr int EB = LD::EB, NV = S::NV, NP = S::NP, NF = S::NF;
    constexpr int NFACE = DIM * NV * NF * EB;
    const Ops1D &ops = *reinterpret_cast<const Ops1D *>(lds);
    double *s_u = lds + LD::U;
    double *s_t = lds + LD::T;
    double *s_fm = lds + LD::FM;
    double *s_fp = lds + LD::FP;
    double *s_ih = lds + LD::IH;
    int *s_k = reinterpret_cast<int *>(lds + LD::INTS);
    {
        const double *src_ops = reinterpret_cast<const double *>(&pk.tab->ops[P]);
        for (int t = threadIdx.x; t < LD::OPS; t += blockDim.x) lds[t] = src_ops[t];
    }
    const int b0 = blk * EB;
    const int ne = min(EB, pk.count - b0);
    const double alpha = (MODE == SRC_AXPY) ? sval(src.alpha) : 0.0;
    const size_t Ne = (size_t)m.Ne;
    for (int t = threadIdx.x; t < EB; t += blockDim.x) s_k[t] = (t < ne) ? pk.list[b0 + t] : 0;
    __syncthreads();
    for (int t = threadIdx.x; t < NV * NP * EB; t += blockDim.x) {
        const int e = t % EB, vi = t / EB;
        s_u[t] = (e < ne) ? load_state<MODE>(src, m, vi / NP, vi % NP, s_k[e], alpha) : 0.0;
    }
    for (int t = threadIdx.x; t < NFACE; t += blockDim.x) {
        const int e = t % EB;
        const int r = t / EB;  // (a * NV + v) * NF + f
        double vt = 0.0, vp = 0.0, vm = 0.0;
        if (e < ne) {
            const size_t idx = ((size_t)(r / NF) * pk.NFM + r % NF) * Ne + s_k[e];
            vt = Jp[idx];
            vp = Fs[idx];
            vm = pk.Fm[idx];
        }
        s_t[t] = vt;
        s_fp[t] = vp;
        s_fm[t] = vm;
    }
    for (int t = threadIdx.x; t < DIM * EB; t += blockDim.x) {
        const int e = t % EB, a = t / EB;
        s_ih[t] = (e < ne) ? pa_inv2h(m, pk, s_k[e], a) : 0.0;
    }
    __syncthreads();
    const int t = threadIdx.x;
    const int e = t % EB, i = t / EB;
    const bool active = (t < NP * EB) && (e < ne);
    double acc[NV];
    divergence<DIM, P, EB, EB>(ops, ph, s_u, s_t, s_fm, s_fp, s_ih, active, e, i, acc);
    // the padding entries: 0 (the inputs' padding is not read)
    const int npad = pk.NpM - NP;
    for (int u = threadIdx.x; u < NV * npad * EB; u += blockDim.x) {
        const int e2 = u % EB, r = u / EB;
        if (e2 >= ne) continue;
        const int v = r / npad, i2 = NP + r % npad;
        o.r[((size_t)v * pk.NpM + i2) * Ne + s_k[e2]] = 0.0;
    }
    if (!active) return;
    const int k = s_k[e];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const double R = -acc[v];
        const size_t idx = ((size_t)v * pk.NpM + i) * Ne + k;
        if (OUT == OUT_R) {
            o.r[idx] = R;
        } else {
            double val = o.sigma * o.vdir[idx] - (R - o.r0[idx]) / (alpha * o.dscale);
            if (o.x) val -= o.x[idx];
            o.r[idx] = val;
        }
    }
}

// One launch per phase for every class: workgroups [boff[P], boff[P + 1])
// take class P (its elements cls[eoff[P] .. eoff[P + 1])), the body is the
// class's own compile-time instantiation and the LDS is carved from one
// dynamic buffer sized for the largest class.
struct PaGrid {
    const int *cls;
    int eoff[kMaxP + 2];
    int boff[kMaxP + 2];
};

__device__ __forceinline__ int pa_class_of(const PaGrid &g, int b) {
    int P = 1;
    while (P < kMaxP && b >= g.boff[P + 1]) ++P;
    return P;
}

template <int DIM, int MODE>
__global__ void __launch_bounds__(DIM == 2 ? 128 : 192) __attribute__((amdgpu_waves_per_eu(4, 8)))
k_pa_faces_all(MeshK m, SrcK src, Phys ph, PaK pk, PaGrid g, double *__restrict__ Jp, double *__restrict__ Fs) {
    extern __shared__ double lds[];
    const int b = xcd_block(blockIdx.x, gridDim.x);
    const int P = pa_class_of(g, b);
    pk.list = g.cls + g.eoff[P];
    pk.count = g.eoff[P + 1] - g.eoff[P];
    const int blk = b - g.boff[P];
    switch (P) {
        case 1: pa_faces_body<DIM, 1, MODE>(m, src, ph, pk, Jp, Fs, blk, lds); break;
        case 2: pa_faces_body<DIM, 2, MODE>(m, src, ph, pk, Jp, Fs, blk, lds); break;
        case 3: pa_faces_body<DIM, 3, MODE>(m, src, ph, pk, Jp, Fs, blk, lds); break;
        case 4: pa_faces_body<DIM, 4, MODE>(m, src, ph, pk, Jp, Fs, blk, lds); break;
        default:
            if constexpr (DIM == 2) pa_faces_body<DIM, 5, MODE>(m, src, ph, pk, Jp, Fs, blk, lds);
            break;
    }
}

template <int DIM, int MODE, int OUT>
__global__ void __launch_bounds__(256) k_pa_volume_all(MeshK m, SrcK src, Phys ph, PaK pk, PaGrid g,
                                                       const double *__restrict__ Jp, const double *__restrict__ Fs,
                                                       OutK o) {
    extern __shared__ double lds[];
    const int b = xcd_block(blockIdx.x, gridDim.x);
    const int P = pa_class_of(g, b);
    pk.list = g.cls + g.eoff[P];
    pk.count = g.eoff[P + 1] - g.eoff[P];
    const int blk = b - g.boff[P];
    switch (P) {
        case 1: pa_volume_body<DIM, 1, MODE, OUT>(m, src, ph, pk, Jp, Fs, o, blk, lds); break;
        case 2: pa_volume_body<DIM, 2, MODE, OUT>(m, src, ph, pk, Jp, Fs, o, blk, lds); break;
        case 3: pa_volume_body<DIM, 3, MODE, OUT>(m, src, ph, pk, Jp, Fs, o, blk, lds); break;
        case 4: pa_volume_body<DIM, 4, MODE, OUT>(m, src, ph, pk, Jp, Fs, o, blk, lds); break;
        default:
            if constexpr (DIM == 2) pa_volume_body<DIM, 5, MODE, OUT>(m, src, ph, pk, Jp, Fs, o, blk, lds);
            break;
    }
}

// ---- EJ blocks of a mixed-degree level by coloured one-sided differences --

__global__ void k_pa_blk_identity(size_t total, int nb, double *__restrict__ B) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    const size_t nn = (size_t)nb * nb;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += stride) {
        const size_t w = t % nn;
        B[t] = (w / nb == w % nb) ? 1.0 : 0.0;
    }
}

__device__ __forceinline__ int elem_colour(const MeshK &m, int k) {
    int c[3];
    coords(m, k, c);
    return (c[0] & 1) | ((c[1] & 1) << 1) | ((c[2] & 1) << 2);
}

// Copy b of a batch of perturbed states: dq plus, on the elements of the
// colour of pair t0 + b, the step of that pair's column (pair t: colour
// t / n_b, column t % n_b; pairs beyond npairs are left unperturbed).
// qB is [nv][NpM][B ne0].
__global__ void k_pa_fd_perturb(MeshK m, const int *__restrict__ Pk, int NpM, int nv, int nb, int B, int t0,
                                int npairs, Phys ph, const double *__restrict__ dq, double *__restrict__ qB) {
    const int ne0 = m.Ne;
    const size_t total = (size_t)nv * NpM * B * ne0;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += stride) {
        const int k = (int)(t % ne0);
        const size_t r = t / ne0;
        const int b = (int)(r % B);
        const int vi = (int)(r / B);
        const double base = dq[(size_t)vi * ne0 + k];
        double val = base;
        const int pair = t0 + b;
        if (pair < npairs && vi == pair % nb && elem_colour(m, k) == pair / nb) {
            const int P = Pk[k];
            const int np = (m.dim == 2) ? P * P : P * P * P;
            if (vi % NpM < np) val = base + fd_step(ph.qinf[vi / NpM], base);
        }
        qB[t] = val;
    }
}

// column j of B_k = sigma e_j - (R_k(q + h e_j) - R_k(q)) / h on the valid
// rows, for the elements perturbed in copy b (pair t0 + b)
__global__ void k_pa_fd_extract(MeshK m, const int *__restrict__ Pk, int NpM, int nb, int B, int t0, int npairs,
                                Phys ph, const double *__restrict__ dq, const double *__restrict__ rB,
                                const double *__restrict__ r0, double sigma, double *__restrict__ Bk) {
    const int ne0 = m.Ne;
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (size_t)B * nb * ne0) return;
    const int k = (int)(t % ne0);
    const size_t r = t / ne0;
    const int row = (int)(r % nb), b = (int)(r / nb);
    const int pair = t0 + b;
    if (pair >= npairs || elem_colour(m, k) != pair / nb) return;
    const int j = pair % nb;
    const int P = Pk[k];
    const int np = (m.dim == 2) ? P * P : P * P * P;
    if (j % NpM >= np || row % NpM >= np) return;
    const double base = dq[(size_t)j * ne0 + k];
    const double hact = (base + fd_step(ph.qinf[j / NpM], base)) - base;
    double val = -(rB[((size_t)row * B + b) * ne0 + k] - r0[(size_t)row * ne0 + k]) / hact;
    if (row == j) val += sigma;
    Bk[(size_t)k * nb * nb + (size_t)j * nb + row] = val;
}

// ---- per-element transfers, indicator and degree update ------------------

// y (=, or += when acc) the per-element L2 projection of x - x0 (x0 optional)
// from Pf[k] + dP to Pt[k] + dP points per direction (dP = 1: degree maps); y2 likewise from x2 (optional).
// One lane per output entry; padding of y is zeroed unless accumulating.
__global__ void k_pa_transfer(int dim, int nv, int Ne, const int *__restrict__ Pf, int NpF, const int *__restrict__ Pt,
                              int NpT, int dP, const PaTables *__restrict__ tab, const double *__restrict__ x,
                              const double *__restrict__ x0, double *__restrict__ y, int acc,
                              const double *__restrict__ x2, double *__restrict__ y2) {
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (size_t)nv * NpT * Ne) return;
    const int k = (int)(t % Ne);
    const int r = (int)(t / Ne);
    const int v = r / NpT, i = r % NpT;
    const int pf = Pf[k] + dP, pt = Pt[k] + dP;
    const int nf = (dim == 2) ? pf * pf : pf * pf * pf, nt = (dim == 2) ? pt * pt : pt * pt * pt;
    if (pf < 1 || pt < 1 || nf > NpF || nt > NpT) {  // a degree beyond the padded layout: no value
        y[t] = __builtin_nan("");
        if (y2) y2[t] = __builtin_nan("");
        return;
    }
    if (i >= nt) {
        if (!acc) {
            y[t] = 0.0;
            if (y2) y2[t] = 0.0;
        }
        return;
    }
    const size_t xb = (size_t)v * NpF * Ne + k;
    double s = 0.0, s2 = 0.0;
    if (pf == pt) {
        s = x[xb + (size_t)i * Ne] - (x0 ? x0[xb + (size_t)i * Ne] : 0.0);
        if (x2) s2 = x2[xb + (size_t)i * Ne];
    } else {
        const int b0 = i % pt, b1 = (i / pt) % pt, b2 = i / (pt * pt);
        for (int i2 = 0; i2 < nf; ++i2) {
            const int a0 = i2 % pf, a1 = (i2 / pf) % pf, a2 = i2 / (pf * pf);
            double c = tab->proj[pf][pt][b0][a0] * tab->proj[pf][pt][b1][a1];
            if (dim == 3) c *= tab->proj[pf][pt][b2][a2];
            const size_t xi = xb + (size_t)i2 * Ne;
            s += c * (x[xi] - (x0 ? x0[xi] : 0.0));
            if (x2) s2 += c * x2[xi];
        }
    }
    y[t] = acc ? y[t] + s : s;
    if (x2) y2[t] = s2;
}

// eta_k = ||s_p - s_{p-1}|| / ||s_p|| of s = q_inf[var] + dq[var]: the energy
// of the Legendre modes whose largest index is p over that of all modes (the
// element's Jacobian cancels).  One lane per element.
__global__ void k_pa_indicator(int dim, int Ne, const int *__restrict__ Pk, int NpM, const PaTables *__restrict__ tab,
                               double qv, const double *__restrict__ s, double *__restrict__ eta) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= Ne) return;
    const int P = Pk[k];
    double u[kMaxNF3 * 4], w[kMaxNF3 * 4];  // 2D: P^2 <= 25; 3D: P^3 <= 64 (p <= 3)
    const int np = (dim == 2) ? P * P : P * P * P;
    for (int i = 0; i < np; ++i) u[i] = qv + s[(size_t)i * Ne + k];
    // modal coefficients, one direction at a time
    const double(*M)[kMaxP] = tab->modal[P];
    const int stride[3] = {1, P, P * P};
    for (int d = 0; d < dim; ++d) {
        const int st = stride[d];
        for (int i = 0; i < np; ++i) {
            const int id = (i / st) % P, base = i - id * st;
            double acc = 0.0;
            for (int j = 0; j < P; ++j) acc += M[id][j] * u[base + j * st];
            w[i] = acc;
        }
        for (int i = 0; i < np; ++i) u[i] = w[i];
    }
    double e_all = 0.0, e_top = 0.0;
    for (int i = 0; i < np; ++i) {
        const int n0 = i % P, n1 = (i / P) % P, n2 = (dim == 3) ? i / (P * P) : 0;
        double nrm = (2.0 / (2.0 * n0 + 1.0)) * (2.0 / (2.0 * n1 + 1.0));
        if (dim == 3) nrm *= 2.0 / (2.0 * n2 + 1.0);
        const double en = nrm * u[i] * u[i];
        e_all += en;
        if (max(n0, max(n1, n2)) == P - 1) e_top += en;
    }
    eta[k] = (e_all > 0.0) ? sqrt(e_top / e_all) : 0.0;
}

// Degree update: p + 1 where eta > nu_max eta_max, p - 1 where
// eta < nu_min eta_max, within [p_min, p_max].  One workgroup.
__global__ void __launch_bounds__(1024) k_pa_adapt(int Ne, const double *__restrict__ eta,
                                                   const int *__restrict__ deg_in, int *__restrict__ deg_out,
                                                   int p_min, int p_max, double nu_max, double nu_min) {
    __shared__ double red[1024];
    double mx = 0.0;
    for (int k = threadIdx.x; k < Ne; k += blockDim.x) mx = fmax(mx, eta[k]);
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    const double emax = red[0];
    for (int k = threadIdx.x; k < Ne; k += blockDim.x) {
        int p = deg_in[k];
        if (eta[k] > nu_max * emax) p += 1;
        if (eta[k] < nu_min * emax) p -= 1;
        deg_out[k] = min(max(p, p_min), p_max);
    }
}

// ---- launchers ------------------------------------------------------------

// The elements one mixed-degree evaluation covers: a level, or fdB
// perturbed copies of it (ids b Ne + k), with the lists and face buffers
// sized for them.
struct PaSet {
    MeshK m;  // the level's mesh; Ne = every id of the set
    int ne0;
    const int *Pk, *cls, *mixed;
    const int *cls_off;  // host
    int nmixed;
    double *Jp, *Fs, *Fm, *Mq, *Mn, *Mg;
};

PaSet pa_level_set(const frpmg_ctx *ctx, const Level &L) {
    const PaLevel &pa = *L.pa;
    return PaSet{ctx->mesh, ctx->mesh.Ne, pa.Pk, pa.cls, pa.mixed, pa.cls_off, pa.nmixed,
                 L.Jp, L.Fs, pa.Fm, pa.Mq, pa.Mn, pa.Mg};
}

PaSet pa_batch_set(const frpmg_ctx *ctx, const Level &L) {
    const PaLevel &pa = *L.pa;
    MeshK m = ctx->mesh;
    m.Ne = ctx->mesh.Ne * pa.fdB;
    return PaSet{m, ctx->mesh.Ne, pa.PkB, pa.clsB, pa.mixedB, pa.clsB_off, pa.nmixed * pa.fdB,
                 pa.JpB, pa.FsB, pa.FmB, pa.MqB, pa.MnB, pa.MgB};
}

template <int DIM>
constexpr int pa_max_p() {
    return DIM == 2 ? 5 : 4;
}

// workgroup ranges of the classes for one phase, and the LDS the largest needs
template <int DIM, bool FACES>
size_t pa_grid(const PaSet &ps, PaGrid &g) {
    g.cls = ps.cls;
    size_t lds = 0;
    int nb = 0;
    auto one = [&](auto Pc) {
        constexpr int P = decltype(Pc)::value;
        constexpr int EB = FACES ? PaFacesLds<DIM, P>::EB : PaVolLds<DIM, P>::EB;
        constexpr int DBL = FACES ? PaFacesLds<DIM, P>::DOUBLES : PaVolLds<DIM, P>::DOUBLES;
        const int cnt = ps.cls_off[P + 1] - ps.cls_off[P];
        g.eoff[P] = ps.cls_off[P];
        g.boff[P] = nb;
        nb += (cnt + EB - 1) / EB;
        if (cnt > 0) lds = std::max(lds, (size_t)DBL * sizeof(double));
    };
    one(std::integral_constant<int, 1>{});
    one(std::integral_constant<int, 2>{});
    one(std::integral_constant<int, 3>{});
    one(std::integral_constant<int, 4>{});
    if constexpr (DIM == 2) one(std::integral_constant<int, 5>{});
    for (int P = pa_max_p<DIM>() + 1; P <= kMaxP + 1; ++P) {
        g.eoff[P] = ps.cls_off[pa_max_p<DIM>() + 1];
        g.boff[P] = nb;
    }
    g.eoff[0] = g.boff[0] = 0;
    return lds;
}

template <int DIM, int MODE, int OUT>
hipError_t pa_run(const frpmg_ctx *ctx, const Level &L, const PaSet &ps, const ResidualArgs &a, hipStream_t s) {
    PaK pk{ps.Pk, nullptr, 0, ps.ne0, L.Np, L.NF, ctx->pa_tab, ps.Fm, ps.Mq, ps.Mn, ps.Mg};
    SrcK src{a.dq, a.v, a.alpha, L.Np};
    PaGrid gf, gv;
    const size_t lf = pa_grid<DIM, true>(ps, gf), lv = pa_grid<DIM, false>(ps, gv);
    const int nf = gf.boff[kMaxP + 1], nv = gv.boff[kMaxP + 1];
    if (nf > 0) {
        hipLaunchKernelGGL((k_pa_faces_all<DIM, MODE>), dim3(nf), dim3(DIM == 2 ? 128 : 192), lf, s, ps.m, src,
                           ctx->phys, pk, gf, ps.Jp, ps.Fs);
    }
    if (ps.nmixed > 0) {
        constexpr int FB = 64 / ((DIM == 2) ? kMaxP : kMaxNF3);
        hipLaunchKernelGGL((k_pa_mortar<DIM>), dim3((ps.nmixed + FB - 1) / FB), dim3(64), 0, s, ps.m, ctx->phys, pk,
                           ps.mixed, ps.nmixed, ps.Fs);
    }
    if (nv > 0) {
        OutK o{a.r, a.r0, a.x, a.v, a.sigma, a.dscale};
        hipLaunchKernelGGL((k_pa_volume_all<DIM, MODE, OUT>), dim3(nv), dim3(256), lv, s, ps.m, src, ctx->phys, pk,
                           gv, ps.Jp, ps.Fs, o);
    }
    return hipGetLastError();
}

template <int DIM>
hipError_t pa_dispatch(const frpmg_ctx *ctx, const Level &L, const PaSet &ps, const ResidualArgs &a,
                       hipStream_t s) {
    if (a.src == SRC_PLAIN && a.out == OUT_R) return pa_run<DIM, SRC_PLAIN, OUT_R>(ctx, L, ps, a, s);
    if (a.src == SRC_AXPY && a.out == OUT_R) return pa_run<DIM, SRC_AXPY, OUT_R>(ctx, L, ps, a, s);
    if (a.src == SRC_AXPY && a.out == OUT_LIN) return pa_run<DIM, SRC_AXPY, OUT_LIN>(ctx, L, ps, a, s);
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_residual(const frpmg_ctx *ctx, int level, const ResidualArgs &a, hipStream_t s) {
    const Level &L = ctx->lv[level];
    if (L.pa) return launch_residual_pa(ctx, level, a, s);
    if (ctx->dim == 2) {
        switch (L.P) {
            case 1: return dispatch_modes<2, 1>(ctx, L, a, nullptr, s);
            case 2: return dispatch_modes<2, 2>(ctx, L, a, nullptr, s);
            case 3: return dispatch_modes<2, 3>(ctx, L, a, nullptr, s);
            case 4: return dispatch_modes<2, 4>(ctx, L, a, nullptr, s);
            case 5: return dispatch_modes<2, 5>(ctx, L, a, nullptr, s);
        }
    } else {
        switch (L.P) {
            case 1: return dispatch_modes<3, 1>(ctx, L, a, nullptr, s);
            case 2: return dispatch_modes<3, 2>(ctx, L, a, nullptr, s);
            case 3: return dispatch_modes<3, 3>(ctx, L, a, nullptr, s);
            case 4: return dispatch_modes<3, 4>(ctx, L, a, nullptr, s);
        }
    }
    return hipErrorInvalidValue;
}

hipError_t launch_ej_form(const frpmg_ctx *ctx, int level, const double *dq, double sigma, hipStream_t s,
                          double *out) {
    const Level &L = ctx->lv[level];
    if (!out) out = L.blk64;
    if (L.pa) return launch_ej_form_pa(ctx, level, dq, sigma, s, out);
    if (!L.fQs || !L.fQp || !L.fSn || !L.fGt || !out || !L.r0) return hipErrorInvalidValue;
    if (ctx->dim == 2) {
        switch (L.P) {
            case 1: return form<2, 1>(ctx, L, dq, sigma, out, s);
            case 2: return form<2, 2>(ctx, L, dq, sigma, out, s);
            case 3: return form<2, 3>(ctx, L, dq, sigma, out, s);
            case 4: return form<2, 4>(ctx, L, dq, sigma, out, s);
            case 5: return form<2, 5>(ctx, L, dq, sigma, out, s);
        }
    } else {
        switch (L.P) {
            case 1: return form<3, 1>(ctx, L, dq, sigma, out, s);
            case 2: return form<3, 2>(ctx, L, dq, sigma, out, s);
            case 3: return form<3, 3>(ctx, L, dq, sigma, out, s);
            case 4: return form<3, 4>(ctx, L, dq, sigma, out, s);
        }
    }
    return hipErrorInvalidValue;
}

hipError_t launch_residual_batch(const frpmg_ctx *ctx, int level, int batch, const double *dq, double *r,
                                 double *Jp, double *Fs, hipStream_t s) {
    const Level &L = ctx->lv[level];
    MeshK m = ctx->mesh;
    if (batch < 1 || (ctx->dim == 3 && batch != 1)) return hipErrorInvalidValue;
    // copy b occupies elements b Ne .. (b + 1) Ne - 1: the third coordinate of
    // a 2D element, which no face or neighbour lookup changes
    const unsigned long long ne = (unsigned long long)m.Ne * (unsigned long long)batch;
    if (ne > 0x7fffffffULL || ne * (unsigned long long)std::max(m.n[0], m.n[1]) >= (1ULL << 40))
        return hipErrorInvalidValue;
    m.Ne = (int)ne;
    if (ctx->dim == 2) m.n[2] = batch;
    ResidualArgs a;
    a.src = SRC_PLAIN;
    a.dq = dq;
    a.out = OUT_R;
    a.r = r;
    if (ctx->dim == 2) {
        switch (L.P) {
            case 1: return run_on<2, 1, SRC_PLAIN, OUT_R>(ctx, L, m, Jp, Fs, a, nullptr, s);
            case 2: return run_on<2, 2, SRC_PLAIN, OUT_R>(ctx, L, m, Jp, Fs, a, nullptr, s);
            case 3: return run_on<2, 3, SRC_PLAIN, OUT_R>(ctx, L, m, Jp, Fs, a, nullptr, s);
            case 4: return run_on<2, 4, SRC_PLAIN, OUT_R>(ctx, L, m, Jp, Fs, a, nullptr, s);
            case 5: return run_on<2, 5, SRC_PLAIN, OUT_R>(ctx, L, m, Jp, Fs, a, nullptr, s);
        }
    } else {
        switch (L.P) {
            case 1: return run_on<3, 1, SRC_PLAIN, OUT_R>(ctx, L, m, Jp, Fs, a, nullptr, s);
            case 2: return run_on<3, 2, SRC_PLAIN, OUT_R>(ctx, L, m, Jp, Fs, a, nullptr, s);
            case 3: return run_on<3, 3, SRC_PLAIN, OUT_R>(ctx, L, m, Jp, Fs, a, nullptr, s);
            case 4: return run_on<3, 4, SRC_PLAIN, OUT_R>(ctx, L, m, Jp, Fs, a, nullptr, s);
        }
    }
    return hipErrorInvalidValue;
}

hipError_t launch_residual_pa(const frpmg_ctx *ctx, int level, const ResidualArgs &a, hipStream_t s) {
    const Level &L = ctx->lv[level];
    if (!L.pa || !ctx->pa_tab || !ctx->pa_tab_host) return hipErrorInvalidValue;
    const PaSet ps = pa_level_set(ctx, L);
    return ctx->dim == 2 ? pa_dispatch<2>(ctx, L, ps, a, s) : pa_dispatch<3>(ctx, L, ps, a, s);
}

hipError_t launch_ej_form_pa(const frpmg_ctx *ctx, int level, const double *dq, double sigma, hipStream_t s,
                             double *out) {
    const Level &L = ctx->lv[level];
    if (!L.pa || !out || !L.r0) return hipErrorInvalidValue;
    const PaLevel &pa = *L.pa;
    const MeshK &m = ctx->mesh;
    for (int a = 0; a < ctx->dim; ++a)
        if (m.n[a] % 2) return hipErrorInvalidValue;
    ResidualArgs a0;
    a0.src = SRC_PLAIN;
    a0.dq = dq;
    a0.out = OUT_R;
    a0.r = L.r0;
    hipError_t err = launch_residual_pa(ctx, level, a0, s);
    if (err != hipSuccess) return err;
    const size_t total = (size_t)m.Ne * L.nb * L.nb;
    hipLaunchKernelGGL(k_pa_blk_identity, dim3(4096), dim3(256), 0, s, total, L.nb, out);
    // (colour, column) pairs, fdB per evaluation of the perturbed copies
    const PaSet ps = pa_batch_set(ctx, L);
    const int B = pa.fdB;
    const int npairs = (1 << ctx->dim) * L.nb;
    const size_t nq = (size_t)ctx->nv * L.Np * B * m.Ne;
    const dim3 gq((unsigned)std::min<size_t>((nq + 255) / 256, 65536));
    const dim3 gx((unsigned)(((size_t)B * L.nb * m.Ne + 255) / 256));
    ResidualArgs ap;
    ap.src = SRC_PLAIN;
    ap.dq = pa.qB;
    ap.out = OUT_R;
    ap.r = pa.rB;
    for (int t0 = 0; t0 < npairs; t0 += B) {
        hipLaunchKernelGGL(k_pa_fd_perturb, gq, dim3(256), 0, s, m, pa.Pk, L.Np, ctx->nv, L.nb, B, t0, npairs,
                           ctx->phys, dq, pa.qB);
        err = ctx->dim == 2 ? pa_dispatch<2>(ctx, L, ps, ap, s) : pa_dispatch<3>(ctx, L, ps, ap, s);
        if (err != hipSuccess) return err;
        hipLaunchKernelGGL(k_pa_fd_extract, gx, dim3(256), 0, s, m, pa.Pk, L.Np, L.nb, B, t0, npairs, ctx->phys,
                           dq, pa.rB, L.r0, sigma, out);
    }
    return hipGetLastError();
}

hipError_t pa_project(const frpmg_ctx *ctx, const int *deg_from, int NpF, const double *x, const int *deg_to, int NpT,
                      double *y, hipStream_t s) {
    if (!ctx->pa_tab) return hipErrorInvalidValue;
    const size_t n = (size_t)ctx->nv * NpT * ctx->mesh.Ne;
    hipLaunchKernelGGL(k_pa_transfer, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, ctx->dim, ctx->nv,
                       ctx->mesh.Ne, deg_from, NpF, deg_to, NpT, 1, ctx->pa_tab, x, nullptr, y, 0, nullptr, nullptr);
    return hipGetLastError();
}

hipError_t pa_transfer(const frpmg_ctx *ctx, int from, int to, const double *x, double *y, const double *x0,
                       bool accumulate, const double *x2, double *y2, hipStream_t s) {
    const Level &A = ctx->lv[from], &B = ctx->lv[to];
    if (!A.pa || !B.pa || !ctx->pa_tab) return hipErrorInvalidValue;
    const size_t n = (size_t)ctx->nv * B.Np * ctx->mesh.Ne;
    hipLaunchKernelGGL(k_pa_transfer, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, ctx->dim, ctx->nv,
                       ctx->mesh.Ne, A.pa->Pk, A.Np, B.pa->Pk, B.Np, 0, ctx->pa_tab, x, x0, y, accumulate ? 1 : 0, x2,
                       y2);
    return hipGetLastError();
}

hipError_t pa_indicator(const frpmg_ctx *ctx, int level, const double *dq, int var, double *eta, hipStream_t s) {
    const Level &L = ctx->lv[level];
    if (!L.pa || var < 0 || var >= ctx->nv) return hipErrorInvalidValue;
    const int Ne = ctx->mesh.Ne;
    hipLaunchKernelGGL(k_pa_indicator, dim3((Ne + 127) / 128), dim3(128), 0, s, ctx->dim, Ne, L.pa->Pk, L.Np,
                       ctx->pa_tab, ctx->phys.qinf[var], dq + (size_t)var * L.Np * Ne, eta);
    return hipGetLastError();
}

hipError_t pa_adapt(const frpmg_ctx *ctx, const double *eta, const int *deg_in, int *deg_out, int p_min, int p_max,
                    double nu_max, double nu_min, hipStream_t s) {
    hipLaunchKernelGGL(k_pa_adapt, dim3(1), dim3(1024), 0, s, ctx->mesh.Ne, eta, deg_in, deg_out, p_min, p_max,
                       nu_max, nu_min);
    return hipGetLastError();
}

}  // namespace frpmg
