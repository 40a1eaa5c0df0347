/*
 * fr_oracle.c -- plain FP64 CPU oracle for the flux-reconstruction (FR)
 * residual of the compressible Navier-Stokes equations, the element-Jacobi
 * (EJ) diagonal blocks built from it, the block LU, and the L2-projection
 * transfer operators between polynomial degrees.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code
 * with the GPU path (no headers, no helpers, no tables).
 *
 * Paper: L. Wang, W. Trojak, F. Witherden, A. Jameson, "Nonlinear p-multigrid
 * preconditioner for implicit time integration of compressible Navier-Stokes
 * equations", arXiv 2202.09733.
 *   - Conservation law dq/dt + div f = 0: Sec. 2.1, Eq. (1).  R(q) is the FR
 *     right-hand side, dq/dt = R(q) (sign as used by the ESDIRK/ROW stage
 *     equations of Sec. 2.1).
 *   - FR itself is only cited in Sec. 2.1; this file fixes one consistent
 *     reading: Gauss-Legendre solution points, Huynh's DG-recovering (Radau)
 *     correction functions, flux-polynomial traces, the original Roe flux
 *     without entropy fix (Sec. 4.2.1), and an LDG viscous flux with the
 *     common solution taken from the +axis element and the common viscous
 *     flux from the -axis element plus a penalty tau*(q_R - q_L).
 *   - Restriction/prolongation: L2 projection with mass matrices on the
 *     standard element, Sec. 3.1 Eqs. (projection) and (prolongation).
 *   - EJ blocks: diagonal blocks of the shifted Jacobian, Sec. 2.2 (element-
 *     Jacobi preconditioner), formed by one-sided finite differences.
 *
 * State convention.  Every state array holds the DEVIATION dq = q - q_inf of
 * the conservative variables from the uniform reference state q_inf, laid out
 * as [nvar][npts][nelem] (element index fastest).  All fluxes are evaluated
 * as f(q) - f(q_inf) through identities that are exact in real arithmetic, so
 * R(0) = 0 exactly and low-Mach states do not lose digits to p_inf.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAXP 8

/* ------------------------------------------------------------------------ */
/* 1D operators on the reference interval [-1, 1]                           */
/* ------------------------------------------------------------------------ */

/* Legendre polynomial L_n(x) and its derivative, by the three-term
 * recurrence (n+1) L_{n+1} = (2n+1) x L_n - n L_{n-1} and
 * L'_{n+1} = L'_{n-1} + (2n+1) L_n. */
static void legendre(int n, double x, double *L, double *dL)
{
    double l0 = 1.0, l1 = x, d0 = 0.0, d1 = 1.0;
    if (n == 0) { *L = 1.0; *dL = 0.0; return; }
    for (int k = 1; k < n; ++k) {
        double l2 = ((2.0 * k + 1.0) * x * l1 - k * l0) / (k + 1.0);
        double d2 = d0 + (2.0 * k + 1.0) * l1;
        l0 = l1; l1 = l2; d0 = d1; d1 = d2;
    }
    *L = l1; *dL = d1;
}

/* Gauss-Legendre nodes (roots of L_P, ascending) and weights. */
void or_gauss_legendre(int P, double *x, double *w)
{
    for (int i = 0; i < P; ++i) {
        double z = -cos(M_PI * (i + 0.75) / (P + 0.5));
        for (int it = 0; it < 100; ++it) {
            double L, dL;
            legendre(P, z, &L, &dL);
            double dz = L / dL;
            z -= dz;
            if (fabs(dz) < 1e-15) break;
        }
        double L, dL;
        legendre(P, z, &L, &dL);
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dL * dL);
    }
}

/* Lagrange basis polynomial l_j on nodes xi, evaluated at x. */
static double lagrange(int P, const double *xi, int j, double x)
{
    double v = 1.0;
    for (int m = 0; m < P; ++m)
        if (m != j) v *= (x - xi[m]) / (xi[j] - xi[m]);
    return v;
}

/* Derivative of l_j at x, by the product rule over the factors. */
static double lagrange_deriv(int P, const double *xi, int j, double x)
{
    double s = 0.0;
    for (int m = 0; m < P; ++m) {
        if (m == j) continue;
        double t = 1.0 / (xi[j] - xi[m]);
        for (int n = 0; n < P; ++n)
            if (n != j && n != m) t *= (x - xi[n]) / (xi[j] - xi[n]);
        s += t;
    }
    return s;
}

typedef struct {
    int P;
    double xi[OR_MAXP], w[OR_MAXP];
    double D[OR_MAXP][OR_MAXP];  /* D[i][j] = l_j'(xi_i) */
    double bm[OR_MAXP];          /* l_j(-1) */
    double bp[OR_MAXP];          /* l_j(+1) */
    double gLd[OR_MAXP];         /* g_L'(xi_i) */
    double gRd[OR_MAXP];         /* g_R'(xi_i) */
} ops1d;

/* Huynh's DG-recovering corrections for degree p = P-1:
 * g_L = ((-1)^p / 2)(L_p - L_{p+1}),  g_R = (1/2)(L_p + L_{p+1}). */
static void make_ops1d(int P, ops1d *o)
{
    int p = P - 1;
    double sgn = (p % 2 == 0) ? 1.0 : -1.0;
    o->P = P;
    or_gauss_legendre(P, o->xi, o->w);
    for (int i = 0; i < P; ++i)
        for (int j = 0; j < P; ++j)
            o->D[i][j] = lagrange_deriv(P, o->xi, j, o->xi[i]);
    for (int j = 0; j < P; ++j) {
        o->bm[j] = lagrange(P, o->xi, j, -1.0);
        o->bp[j] = lagrange(P, o->xi, j, 1.0);
    }
    for (int i = 0; i < P; ++i) {
        double Lp, dLp, Lq, dLq;
        legendre(p, o->xi[i], &Lp, &dLp);
        legendre(p + 1, o->xi[i], &Lq, &dLq);
        o->gLd[i] = 0.5 * sgn * (dLp - dLq);
        o->gRd[i] = 0.5 * (dLp + dLq);
    }
}

/* Export of the 1D operators for tests.  out receives, in order:
 * xi[P], w[P], D[P*P] (row i = node), bm[P], bp[P], gLd[P], gRd[P]. */
void or_ops1d(int P, double *out)
{
    ops1d o;
    make_ops1d(P, &o);
    double *q = out;
    for (int i = 0; i < P; ++i) *q++ = o.xi[i];
    for (int i = 0; i < P; ++i) *q++ = o.w[i];
    for (int i = 0; i < P; ++i)
        for (int j = 0; j < P; ++j) *q++ = o.D[i][j];
    for (int i = 0; i < P; ++i) *q++ = o.bm[i];
    for (int i = 0; i < P; ++i) *q++ = o.bp[i];
    for (int i = 0; i < P; ++i) *q++ = o.gLd[i];
    for (int i = 0; i < P; ++i) *q++ = o.gRd[i];
}

/* Solve the small dense system A X = B (A n x n, B n x m, row-major) by
 * Gaussian elimination with partial pivoting; X overwrites B. */
static void dense_solve(int n, int m, double *A, double *B)
{
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (fabs(A[r * n + c]) > fabs(A[piv * n + c])) piv = r;
        if (piv != c) {
            for (int j = 0; j < n; ++j) { double t = A[c*n+j]; A[c*n+j] = A[piv*n+j]; A[piv*n+j] = t; }
            for (int j = 0; j < m; ++j) { double t = B[c*m+j]; B[c*m+j] = B[piv*m+j]; B[piv*m+j] = t; }
        }
        for (int r = c + 1; r < n; ++r) {
            double f = A[r * n + c] / A[c * n + c];
            for (int j = c; j < n; ++j) A[r * n + j] -= f * A[c * n + j];
            for (int j = 0; j < m; ++j) B[r * m + j] -= f * B[c * m + j];
        }
    }
    for (int c = n - 1; c >= 0; --c)
        for (int j = 0; j < m; ++j) {
            double s = B[c * m + j];
            for (int k = c + 1; k < n; ++k) s -= A[c * n + k] * B[k * m + j];
            B[c * m + j] = s / A[c * n + c];
        }
}

/* 1D restriction Gamma = (M^{p1})^{-1} M^{p1 p0}  (P1 x P0) and prolongation
 * Pi = (M^{p0})^{-1} M^{p0 p1}  (P0 x P1), with M_ij = int l_i l_j on [-1,1]
 * integrated exactly by a Gauss-Legendre rule of P0 + P1 points
 * (Sec. 3.1, Eqs. (projection) and (prolongation)). */
void or_transfer1d(int P0, int P1, double *Gam, double *Pi)
{
    double x0[OR_MAXP], w0[OR_MAXP], x1[OR_MAXP], w1[OR_MAXP];
    double xq[2 * OR_MAXP], wq[2 * OR_MAXP];
    int Q = P0 + P1;
    or_gauss_legendre(P0, x0, w0);
    or_gauss_legendre(P1, x1, w1);
    or_gauss_legendre(Q, xq, wq);
    double M0[OR_MAXP * OR_MAXP], M1[OR_MAXP * OR_MAXP];
    double M10[OR_MAXP * OR_MAXP], M01[OR_MAXP * OR_MAXP];
    for (int i = 0; i < P0; ++i)
        for (int j = 0; j < P0; ++j) {
            double s = 0.0;
            for (int q = 0; q < Q; ++q)
                s += wq[q] * lagrange(P0, x0, i, xq[q]) * lagrange(P0, x0, j, xq[q]);
            M0[i * P0 + j] = s;
        }
    for (int i = 0; i < P1; ++i)
        for (int j = 0; j < P1; ++j) {
            double s = 0.0;
            for (int q = 0; q < Q; ++q)
                s += wq[q] * lagrange(P1, x1, i, xq[q]) * lagrange(P1, x1, j, xq[q]);
            M1[i * P1 + j] = s;
        }
    for (int i = 0; i < P1; ++i)
        for (int j = 0; j < P0; ++j) {
            double s = 0.0;
            for (int q = 0; q < Q; ++q)
                s += wq[q] * lagrange(P1, x1, i, xq[q]) * lagrange(P0, x0, j, xq[q]);
            M10[i * P0 + j] = s;
            M01[j * P1 + i] = s;
        }
    memcpy(Gam, M10, sizeof(double) * P1 * P0);
    dense_solve(P1, P0, M1, Gam);
    memcpy(Pi, M01, sizeof(double) * P0 * P1);
    dense_solve(P0, P1, M0, Pi);
}

/* ------------------------------------------------------------------------ */
/* Mesh and pointwise physics                                                */
/* ------------------------------------------------------------------------ */

typedef struct {
    int dim;            /* 2 or 3 */
    int P;              /* points per direction, p + 1 */
    int n[3];           /* elements per axis (periodic) */
    const double *h[3]; /* element widths along each axis: n[a] entries */
    double gamma, mu, Pr, tau;
    double qinf[5];     /* conservative reference state (rho, rho u.., E) */
} or_mesh;

static int mesh_ne(const or_mesh *m)
{
    return m->n[0] * m->n[1] * (m->dim == 3 ? m->n[2] : 1);
}

static int ipow(int b, int e) { int r = 1; while (e--) r *= b; return r; }

static void elem_coords(const or_mesh *m, int k, int c[3])
{
    c[0] = k % m->n[0];
    c[1] = (k / m->n[0]) % m->n[1];
    c[2] = (m->dim == 3) ? k / (m->n[0] * m->n[1]) : 0;
}

static int elem_index(const or_mesh *m, const int c[3])
{
    return c[0] + m->n[0] * (c[1] + m->n[1] * c[2]);
}

/* Periodic neighbour of element k at offset s (+1 or -1) along axis a. */
static int neighbour(const or_mesh *m, int k, int a, int s)
{
    int c[3];
    elem_coords(m, k, c);
    c[a] = (c[a] + s + m->n[a]) % m->n[a];
    return elem_index(m, c);
}

/* Local point index of the point at position j along axis a on the line
 * through face point f (face points enumerate the other axes, lowest axis
 * fastest); local points are i = i0 + P (i1 + P i2). */
static int line_point(int dim, int P, int a, int f, int j)
{
    int idx[3] = {0, 0, 0};
    for (int b = 0; b < dim; ++b) {
        if (b == a) idx[b] = j;
        else { idx[b] = f % P; f /= P; }
    }
    return idx[0] + P * (idx[1] + P * idx[2]);
}

/* Face point index and position along axis a of local point i. */
static void point_split(int dim, int P, int a, int i, int *f, int *ia)
{
    int idx[3] = {i % P, (i / P) % P, (dim == 3) ? i / (P * P) : 0};
    int ff = 0, mul = 1;
    for (int b = 0; b < dim; ++b) {
        if (b == a) continue;
        ff += idx[b] * mul;
        mul *= P;
    }
    *f = ff;
    *ia = idx[a];
}

typedef struct {
    double rho, u[3], E, p, H;        /* absolute values */
    double drho, dm[3], du[3], dE, dp; /* deviations from the reference state */
} state_t;

/* Primitive variables from a conservative deviation dq (length dim+2). */
static void primitives(int dim, double gam, const double *qinf, const double *dq, state_t *s)
{
    double rinf = qinf[0], Einf = qinf[dim + 1];
    s->drho = dq[0];
    s->rho = rinf + dq[0];
    double dK2 = 0.0, kin2inf = 0.0;
    for (int b = 0; b < 3; ++b) { s->u[b] = 0.0; s->du[b] = 0.0; s->dm[b] = 0.0; }
    for (int b = 0; b < dim; ++b) {
        double minf = qinf[1 + b];
        double uinf = minf / rinf;
        s->dm[b] = dq[1 + b];
        s->u[b] = (minf + dq[1 + b]) / s->rho;
        /* u - u_inf = (dm - u_inf drho) / rho, exact in real arithmetic */
        s->du[b] = (dq[1 + b] - uinf * dq[0]) / s->rho;
        /* m.u - m_inf.u_inf = dm.u + m_inf.du */
        dK2 += dq[1 + b] * s->u[b] + minf * s->du[b];
        kin2inf += minf * uinf;
    }
    double pinf = (gam - 1.0) * (Einf - 0.5 * kin2inf);
    s->dE = dq[dim + 1];
    s->E = Einf + s->dE;
    s->dp = (gam - 1.0) * (s->dE - 0.5 * dK2);
    s->p = pinf + s->dp;
    s->H = (s->E + s->p) / s->rho;
}

/* Inviscid flux deviation f_a(q) - f_a(q_inf) along axis a. */
static void inviscid_dflux(int dim, int a, const double *qinf, const state_t *s, double *F)
{
    double rinf = qinf[0];
    F[0] = s->dm[a];
    for (int b = 0; b < dim; ++b)
        F[1 + b] = s->dm[a] * s->u[b] + qinf[1 + a] * s->du[b] + (a == b ? s->dp : 0.0);
    F[dim + 1] = s->du[a] * (s->E + s->p) + (qinf[1 + a] / rinf) * (s->dE + s->dp);
}

/* Viscous flux along axis a: (0, tau_a., u.tau_a + (mu gamma / Pr) de/dx_a),
 * constant viscosity, Stokes hypothesis.  grad[c][v] = d q_v / d x_c. */
static void viscous_flux(int dim, int a, double gam, double mu, double Pr,
                         const state_t *s, double grad[3][5], double *F)
{
    int nv = dim + 2;
    double dudx[3][3]; /* dudx[b][c] = d u_b / d x_c */
    double dedx[3];
    double eE = s->E / s->rho;
    for (int c = 0; c < dim; ++c) {
        double kin = 0.0;
        for (int b = 0; b < dim; ++b) {
            dudx[b][c] = (grad[c][1 + b] - s->u[b] * grad[c][0]) / s->rho;
        }
        for (int b = 0; b < dim; ++b) kin += s->u[b] * dudx[b][c];
        dedx[c] = (grad[c][nv - 1] - eE * grad[c][0]) / s->rho - kin;
    }
    double div = 0.0;
    for (int b = 0; b < dim; ++b) div += dudx[b][b];
    double work = 0.0;
    F[0] = 0.0;
    for (int b = 0; b < dim; ++b) {
        double t = mu * (dudx[a][b] + dudx[b][a]) - (a == b ? (2.0 / 3.0) * mu * div : 0.0);
        F[1 + b] = t;
        work += s->u[b] * t;
    }
    F[nv - 1] = work + (mu * gam / Pr) * dedx[a];
}

/* Original Roe flux (no entropy fix) along axis a, returned as the deviation
 * from f_a(q_inf):  (1/2)(df(q_L) + df(q_R)) - (1/2) sum_k |lambda_k| alpha_k r_k. */
static void roe_dflux(int dim, int a, double gam, const double *qinf,
                      const double *dqL, const double *dqR, double *F)
{
    int nv = dim + 2;
    state_t L, R;
    primitives(dim, gam, qinf, dqL, &L);
    primitives(dim, gam, qinf, dqR, &R);
    double FL[5], FRt[5];
    inviscid_dflux(dim, a, qinf, &L, FL);
    inviscid_dflux(dim, a, qinf, &R, FRt);

    double sL = sqrt(L.rho), sR = sqrt(R.rho);
    double rt = sL * sR;
    double ut[3] = {0, 0, 0}, q2 = 0.0;
    for (int b = 0; b < dim; ++b) {
        ut[b] = (sL * L.u[b] + sR * R.u[b]) / (sL + sR);
        q2 += ut[b] * ut[b];
    }
    double Ht = (sL * L.H + sR * R.H) / (sL + sR);
    double c2 = (gam - 1.0) * (Ht - 0.5 * q2);
    double ct = sqrt(c2);
    double un = ut[a];

    double dr = R.drho - L.drho;
    double dP = R.dp - L.dp;
    double dU[3] = {0, 0, 0};
    for (int b = 0; b < dim; ++b) dU[b] = R.du[b] - L.du[b];
    double dUn = dU[a];

    double a1 = (dP - rt * ct * dUn) / (2.0 * c2);
    double a3 = (dP + rt * ct * dUn) / (2.0 * c2);
    double a2 = dr - dP / c2;
    double l1 = fabs(un - ct), l2 = fabs(un), l3 = fabs(un + ct);

    double D[5];
    D[0] = l1 * a1 + l2 * a2 + l3 * a3;
    double utdu = 0.0;
    for (int b = 0; b < dim; ++b) {
        double nb = (a == b) ? 1.0 : 0.0;
        double shear = dU[b] - nb * dUn;
        D[1 + b] = l1 * a1 * (ut[b] - ct * nb) + l2 * a2 * ut[b] + l3 * a3 * (ut[b] + ct * nb)
                 + l2 * rt * shear;
        utdu += ut[b] * dU[b];
    }
    D[nv - 1] = l1 * a1 * (Ht - un * ct) + l2 * a2 * 0.5 * q2 + l3 * a3 * (Ht + un * ct)
              + l2 * rt * (utdu - un * dUn);
    for (int v = 0; v < nv; ++v) F[v] = 0.5 * (FL[v] + FRt[v]) - 0.5 * D[v];
}

/* Exports of the pointwise physics, for tests. */
void or_inviscid_dflux(int dim, int a, double gam, const double *qinf, const double *dq, double *F)
{
    state_t s;
    primitives(dim, gam, qinf, dq, &s);
    inviscid_dflux(dim, a, qinf, &s, F);
}

void or_roe_dflux(int dim, int a, double gam, const double *qinf,
                  const double *dqL, const double *dqR, double *F)
{
    roe_dflux(dim, a, gam, qinf, dqL, dqR, F);
}

/* grad is [dim][dim+2], row c = d/dx_c. */
void or_viscous_flux(int dim, int a, double gam, double mu, double Pr,
                     const double *qinf, const double *dq, const double *grad, double *F)
{
    state_t s;
    double g[3][5];
    primitives(dim, gam, qinf, dq, &s);
    for (int c = 0; c < dim; ++c)
        for (int v = 0; v < dim + 2; ++v) g[c][v] = grad[c * (dim + 2) + v];
    viscous_flux(dim, a, gam, mu, Pr, &s, g, F);
}

/* ------------------------------------------------------------------------ */
/* FR residual                                                               */
/* ------------------------------------------------------------------------ */

/* r = R(dq) on the whole mesh.  Returns 0, or -2 on allocation failure. */
int or_residual(const or_mesh *m, const double *dq, double *r)
{
    const int dim = m->dim, P = m->P, nv = dim + 2;
    const int Ne = mesh_ne(m), Np = ipow(P, dim), NF = ipow(P, dim - 1);
    ops1d o;
    make_ops1d(P, &o);

    /* helpers to index [..][v][pt][k] arrays */
#define QV(arr, v, i, k) (arr)[((size_t)(v) * Np + (i)) * Ne + (k)]
#define TR(arr, a, v, f, k) (arr)[(((size_t)(a) * nv + (v)) * NF + (f)) * Ne + (k)]
#define GR(arr, c, v, i, k) (arr)[(((size_t)(c) * nv + (v)) * Np + (i)) * Ne + (k)]
#define GT(arr, a, c, v, f, k) (arr)[((((size_t)(a) * dim + (c)) * nv + (v)) * NF + (f)) * Ne + (k)]

    size_t ntr = (size_t)dim * nv * NF * Ne;
    size_t ngr = (size_t)dim * nv * Np * Ne;
    double *Tm = malloc(sizeof(double) * ntr);
    double *Tp = malloc(sizeof(double) * ntr);
    double *G = malloc(sizeof(double) * ngr);
    double *GTp = malloc(sizeof(double) * ntr * dim);
    double *Fl = malloc(sizeof(double) * ngr);
    double *FTm = malloc(sizeof(double) * ntr);
    double *FTp = malloc(sizeof(double) * ntr);
    double *Fs = malloc(sizeof(double) * ntr);
    if (!Tm || !Tp || !G || !GTp || !Fl || !FTm || !FTp || !Fs) {
        free(Tm); free(Tp); free(G); free(GTp); free(Fl); free(FTm); free(FTp); free(Fs);
        return -2;
    }

    /* (1) traces of the solution at both ends of every line */
    for (int k = 0; k < Ne; ++k)
        for (int a = 0; a < dim; ++a)
            for (int v = 0; v < nv; ++v)
                for (int f = 0; f < NF; ++f) {
                    double sm = 0.0, sp = 0.0;
                    for (int j = 0; j < P; ++j) {
                        double q = QV(dq, v, line_point(dim, P, a, f, j), k);
                        sm += o.bm[j] * q;
                        sp += o.bp[j] * q;
                    }
                    TR(Tm, a, v, f, k) = sm;
                    TR(Tp, a, v, f, k) = sp;
                }

    /* (2) corrected gradient: the common solution at a face is the trace of
     * the element on the +axis side, so only the + end carries a correction */
    for (int k = 0; k < Ne; ++k) {
        int ck[3];
        elem_coords(m, k, ck);
        for (int c = 0; c < dim; ++c) {
            int kp = neighbour(m, k, c, +1);
            double jac = 2.0 / m->h[c][ck[c]];
            for (int v = 0; v < nv; ++v)
                for (int i = 0; i < Np; ++i) {
                    int f, ic;
                    point_split(dim, P, c, i, &f, &ic);
                    double s = 0.0;
                    for (int j = 0; j < P; ++j)
                        s += o.D[ic][j] * QV(dq, v, line_point(dim, P, c, f, j), k);
                    s += (TR(Tm, c, v, f, kp) - TR(Tp, c, v, f, k)) * o.gRd[ic];
                    GR(G, c, v, i, k) = jac * s;
                }
        }
    }

    /* (3) traces of every gradient component at the + end of each axis */
    for (int k = 0; k < Ne; ++k)
        for (int a = 0; a < dim; ++a)
            for (int c = 0; c < dim; ++c)
                for (int v = 0; v < nv; ++v)
                    for (int f = 0; f < NF; ++f) {
                        double s = 0.0;
                        for (int j = 0; j < P; ++j)
                            s += o.bp[j] * GR(G, c, v, line_point(dim, P, a, f, j), k);
                        GT(GTp, a, c, v, f, k) = s;
                    }

    /* (4) pointwise flux deviation f_a = (f^I_a - f^I_a(q_inf)) - f^V_a */
    for (int k = 0; k < Ne; ++k)
        for (int i = 0; i < Np; ++i) {
            double q[5], grad[3][5];
            state_t s;
            for (int v = 0; v < nv; ++v) q[v] = QV(dq, v, i, k);
            for (int c = 0; c < dim; ++c)
                for (int v = 0; v < nv; ++v) grad[c][v] = GR(G, c, v, i, k);
            primitives(dim, m->gamma, m->qinf, q, &s);
            for (int a = 0; a < dim; ++a) {
                double FI[5], FV[5];
                inviscid_dflux(dim, a, m->qinf, &s, FI);
                viscous_flux(dim, a, m->gamma, m->mu, m->Pr, &s, grad, FV);
                for (int v = 0; v < nv; ++v) GR(Fl, a, v, i, k) = FI[v] - FV[v];
            }
        }

    /* (5) traces of the flux polynomial along its own axis */
    for (int k = 0; k < Ne; ++k)
        for (int a = 0; a < dim; ++a)
            for (int v = 0; v < nv; ++v)
                for (int f = 0; f < NF; ++f) {
                    double sm = 0.0, sp = 0.0;
                    for (int j = 0; j < P; ++j) {
                        double fl = GR(Fl, a, v, line_point(dim, P, a, f, j), k);
                        sm += o.bm[j] * fl;
                        sp += o.bp[j] * fl;
                    }
                    TR(FTm, a, v, f, k) = sm;
                    TR(FTp, a, v, f, k) = sp;
                }

    /* (6) common flux on the + face of every element (face shared with the
     * +axis neighbour): Roe - [f^V(q_L, grad q_L) + tau (q_R - q_L)] */
    for (int k = 0; k < Ne; ++k)
        for (int a = 0; a < dim; ++a) {
            int kp = neighbour(m, k, a, +1);
            for (int f = 0; f < NF; ++f) {
                double qL[5], qR[5], Fr[5], FV[5], grad[3][5];
                state_t sL;
                for (int v = 0; v < nv; ++v) {
                    qL[v] = TR(Tp, a, v, f, k);
                    qR[v] = TR(Tm, a, v, f, kp);
                }
                for (int c = 0; c < dim; ++c)
                    for (int v = 0; v < nv; ++v) grad[c][v] = GT(GTp, a, c, v, f, k);
                roe_dflux(dim, a, m->gamma, m->qinf, qL, qR, Fr);
                primitives(dim, m->gamma, m->qinf, qL, &sL);
                viscous_flux(dim, a, m->gamma, m->mu, m->Pr, &sL, grad, FV);
                for (int v = 0; v < nv; ++v)
                    TR(Fs, a, v, f, k) = Fr[v] - (FV[v] + m->tau * (qR[v] - qL[v]));
            }
        }

    /* (7) R = -sum_a (2/h_a) [D f_a + (F*_- - f^-) g_L' + (F*_+ - f^+) g_R'] */
    for (int k = 0; k < Ne; ++k) {
        int ck[3];
        elem_coords(m, k, ck);
        for (int v = 0; v < nv; ++v)
            for (int i = 0; i < Np; ++i) {
                double acc = 0.0;
                for (int a = 0; a < dim; ++a) {
                    int km = neighbour(m, k, a, -1);
                    int f, ia;
                    point_split(dim, P, a, i, &f, &ia);
                    double s = 0.0;
                    for (int j = 0; j < P; ++j)
                        s += o.D[ia][j] * GR(Fl, a, v, line_point(dim, P, a, f, j), k);
                    s += (TR(Fs, a, v, f, km) - TR(FTm, a, v, f, k)) * o.gLd[ia];
                    s += (TR(Fs, a, v, f, k) - TR(FTp, a, v, f, k)) * o.gRd[ia];
                    acc += (2.0 / m->h[a][ck[a]]) * s;
                }
                QV(r, v, i, k) = -acc;
            }
    }
#undef QV
#undef TR
#undef GR
#undef GT
    free(Tm); free(Tp); free(G); free(GTp); free(Fl); free(FTm); free(FTp); free(Fs);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Element-Jacobi blocks                                                     */
/* ------------------------------------------------------------------------ */

/* B_k = sigma I - dR_k/dq_k for every element k, by one-sided differences
 * of R per column j of the block, with step h_j = 1e-7 max(1, |q_j|) where
 * q_j = q_inf + dq_j is the absolute value; the step actually taken is the
 * representable difference (dq_j + h_j) - dq_j.
 *
 * Elements whose coordinates agree in parity along every axis (one of 2^dim
 * colours) lie outside each other's residual stencil (offsets in {-1,0,1}^dim),
 * so all elements of one colour are perturbed in the same residual
 * evaluation; R_k then equals, bit for bit, the residual of a state in which
 * only element k was perturbed.  Requires an even element count per axis.
 *
 * r0 = R(dq).  B is [Ne][nb][nb], row-major per block: B[k][row][col] with
 * local DOF index v*Np + i.  Returns 0, -1 on odd element counts, -2 on
 * allocation failure. */
int or_ej_blocks(const or_mesh *m, const double *dq, const double *r0, double sigma, double *B)
{
    const int dim = m->dim, nv = dim + 2;
    const int Ne = mesh_ne(m), Np = ipow(m->P, dim), nb = nv * Np;
    for (int a = 0; a < dim; ++a)
        if (m->n[a] % 2 != 0) return -1;
    size_t N = (size_t)nv * Np * Ne;
    double *qp = malloc(sizeof(double) * N);
    double *rp = malloc(sizeof(double) * N);
    double *hk = malloc(sizeof(double) * Ne);
    int *col = malloc(sizeof(int) * Ne);
    if (!qp || !rp || !hk || !col) { free(qp); free(rp); free(hk); free(col); return -2; }
    for (int k = 0; k < Ne; ++k) {
        int c[3];
        elem_coords(m, k, c);
        col[k] = (c[0] & 1) | ((c[1] & 1) << 1) | ((c[2] & 1) << 2);
    }
    int ncol = 1 << dim;
    for (int colour = 0; colour < ncol; ++colour)
        for (int j = 0; j < nb; ++j) {
            int jv = j / Np, ji = j % Np;
            memcpy(qp, dq, sizeof(double) * N);
            for (int k = 0; k < Ne; ++k) {
                if (col[k] != colour) continue;
                size_t idx = ((size_t)jv * Np + ji) * Ne + k;
                double hj = 1e-7 * fmax(1.0, fabs(m->qinf[jv] + dq[idx]));
                qp[idx] = dq[idx] + hj;
                hk[k] = qp[idx] - dq[idx];
            }
            int rc = or_residual(m, qp, rp);
            if (rc) { free(qp); free(rp); free(hk); free(col); return rc; }
            for (int k = 0; k < Ne; ++k) {
                if (col[k] != colour) continue;
                double *Bk = B + (size_t)k * nb * nb;
                for (int row = 0; row < nb; ++row) {
                    size_t idx = (size_t)row * Ne + k; /* row = v*Np + i */
                    Bk[(size_t)row * nb + j] = (row == j ? sigma : 0.0) - (rp[idx] - r0[idx]) / hk[k];
                }
            }
        }
    free(qp); free(rp); free(hk); free(col);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Block LU with partial pivoting (LAPACK getrf semantics)                   */
/* ------------------------------------------------------------------------ */

/* In-place LU of nblk row-major n x n blocks; piv[k*n + c] = pivot row chosen
 * at column c (largest |a|, first index on ties).  Returns 0, or -4 if an
 * exact zero pivot occurs (the factor is still completed where possible). */
int or_lu_factor_batch(int nblk, int n, double *A, int32_t *piv)
{
    int status = 0;
    for (int b = 0; b < nblk; ++b) {
        double *M = A + (size_t)b * n * n;
        int32_t *pv = piv + (size_t)b * n;
        for (int c = 0; c < n; ++c) {
            int p = c;
            double best = fabs(M[(size_t)c * n + c]);
            for (int r = c + 1; r < n; ++r) {
                double v = fabs(M[(size_t)r * n + c]);
                if (v > best) { best = v; p = r; }
            }
            pv[c] = p;
            if (p != c)
                for (int j = 0; j < n; ++j) {
                    double t = M[(size_t)c * n + j];
                    M[(size_t)c * n + j] = M[(size_t)p * n + j];
                    M[(size_t)p * n + j] = t;
                }
            double d = M[(size_t)c * n + c];
            if (d == 0.0) { status = -4; continue; }
            for (int r = c + 1; r < n; ++r) {
                double l = M[(size_t)r * n + c] / d;
                M[(size_t)r * n + c] = l;
                for (int j = c + 1; j < n; ++j) M[(size_t)r * n + j] -= l * M[(size_t)c * n + j];
            }
        }
    }
    return status;
}

/* Solve with the factors of or_lu_factor_batch.  x and y are state arrays in
 * the [nvar][npts][nelem] layout, so block k's right-hand side entry j sits at
 * x[j * nblk + k]. */
void or_lu_solve_batch(int nblk, int n, const double *LU, const int32_t *piv,
                       const double *x, double *y)
{
    double *t = malloc(sizeof(double) * n);
    for (int b = 0; b < nblk; ++b) {
        const double *M = LU + (size_t)b * n * n;
        const int32_t *pv = piv + (size_t)b * n;
        for (int j = 0; j < n; ++j) t[j] = x[(size_t)j * nblk + b];
        for (int c = 0; c < n; ++c) {
            int p = pv[c];
            if (p != c) { double s = t[c]; t[c] = t[p]; t[p] = s; }
        }
        for (int r = 0; r < n; ++r) {
            double s = t[r];
            for (int j = 0; j < r; ++j) s -= M[(size_t)r * n + j] * t[j];
            t[r] = s;
        }
        for (int r = n - 1; r >= 0; --r) {
            double s = t[r];
            for (int j = r + 1; j < n; ++j) s -= M[(size_t)r * n + j] * t[j];
            t[r] = s / M[(size_t)r * n + r];
        }
        for (int j = 0; j < n; ++j) y[(size_t)j * nblk + b] = t[j];
    }
    free(t);
}

/* ------------------------------------------------------------------------ */
/* Mixed polynomial degrees (p-adaptation, Sec. 3.3)                         */
/* ------------------------------------------------------------------------ */

/* Element k carries degree deg[k] (P_k = deg[k] + 1 points per direction,
 * P_k <= m->P).  States are stored padded, [nvar][m->P^dim][nelem]: element k
 * uses local points i < P_k^dim numbered i = i0 + P_k (i1 + P_k i2); the
 * entries beyond are ignored on input and written as zero.
 *
 * The paper leaves the coupling of elements of different degree to its
 * reference on p-adaptation; this oracle fixes the following reading.  At a
 * face between the -axis element L and the +axis element R:
 *   - the common solution is R's trace, as in the uniform scheme; L sees it
 *     through the L2 projection onto L's face polynomials (exact
 *     interpolation when P_L >= P_R);
 *   - the common flux is formed at the Gauss-Legendre points of the larger
 *     of the two degrees (the mortar), from both traces and L's gradient
 *     trace carried there by L2 projection (exact for the lower side), and
 *     is returned to each side's face points by L2 projection (which keeps
 *     its integral over the face, so the scheme stays conservative).
 * Every face map is the tensor product over the face directions of the 1D
 * L2 projection between the two point sets; with equal degrees no map is
 * applied and every operation is that of or_residual, so a uniform degree
 * map reproduces or_residual bit for bit. */

/* T[b * Pa + a]: 1D L2 projection from the Pa-point to the Pb-point space. */
static void proj1d(int Pa, int Pb, double *T)
{
    double Pi[OR_MAXP * OR_MAXP];
    or_transfer1d(Pa, Pb, T, Pi);
}

/* y[fb] = sum_fa T_face[fb][fa] x[fa] between faces of Pa and Pb points per
 * direction (dim - 1 directions, first fastest); xs, ys strides. */
static void face_map(int dim, int Pa, int Pb, const double *T, const double *x, size_t xs,
                     double *y, size_t ys)
{
    int nfa = ipow(Pa, dim - 1), nfb = ipow(Pb, dim - 1);
    for (int fb = 0; fb < nfb; ++fb) {
        int b0 = fb % Pb, b1 = fb / Pb;
        double s = 0.0;
        for (int fa = 0; fa < nfa; ++fa) {
            int a0 = fa % Pa, a1 = fa / Pa;
            double c = T[b0 * Pa + a0];
            if (dim == 3) c *= T[b1 * Pa + a1];
            s += c * x[(size_t)fa * xs];
        }
        y[(size_t)fb * ys] = s;
    }
}

int or_residual_pa(const or_mesh *m, const int *deg, const double *dq, double *r)
{
    const int dim = m->dim, nv = dim + 2, PM = m->P;
    const int Ne = mesh_ne(m), NpM = ipow(PM, dim), NFM = ipow(PM, dim - 1);
    ops1d o[OR_MAXP + 1];
    for (int P = 1; P <= PM; ++P) make_ops1d(P, &o[P]);
    for (int k = 0; k < Ne; ++k)
        if (deg[k] < 0 || deg[k] + 1 > PM) return -3;

#define PQ(arr, v, i, k) (arr)[((size_t)(v) * NpM + (i)) * Ne + (k)]
#define PT(arr, a, v, f, k) (arr)[(((size_t)(a) * nv + (v)) * NFM + (f)) * Ne + (k)]
#define PG(arr, c, v, i, k) (arr)[(((size_t)(c) * nv + (v)) * NpM + (i)) * Ne + (k)]
#define PGT(arr, a, c, v, f, k) (arr)[((((size_t)(a) * dim + (c)) * nv + (v)) * NFM + (f)) * Ne + (k)]

    size_t ntr = (size_t)dim * nv * NFM * Ne;
    size_t ngr = (size_t)dim * nv * NpM * Ne;
    double *Tm = calloc(ntr, sizeof(double)), *Tp = calloc(ntr, sizeof(double));
    double *Qs = calloc(ntr, sizeof(double));
    double *G = calloc(ngr, sizeof(double)), *GTp = calloc(ntr * dim, sizeof(double));
    double *Fl = calloc(ngr, sizeof(double));
    double *FTm = calloc(ntr, sizeof(double)), *FTp = calloc(ntr, sizeof(double));
    double *Fsp = calloc(ntr, sizeof(double)), *Fsm = calloc(ntr, sizeof(double));
    if (!Tm || !Tp || !Qs || !G || !GTp || !Fl || !FTm || !FTp || !Fsp || !Fsm) {
        free(Tm); free(Tp); free(Qs); free(G); free(GTp); free(Fl); free(FTm); free(FTp); free(Fsp); free(Fsm);
        return -2;
    }

    /* (1) own traces at both ends of every line, at the element's own points */
    for (int k = 0; k < Ne; ++k) {
        const int P = deg[k] + 1, NF = ipow(P, dim - 1);
        for (int a = 0; a < dim; ++a)
            for (int v = 0; v < nv; ++v)
                for (int f = 0; f < NF; ++f) {
                    double sm = 0.0, sp = 0.0;
                    for (int j = 0; j < P; ++j) {
                        double q = PQ(dq, v, line_point(dim, P, a, f, j), k);
                        sm += o[P].bm[j] * q;
                        sp += o[P].bp[j] * q;
                    }
                    PT(Tm, a, v, f, k) = sm;
                    PT(Tp, a, v, f, k) = sp;
                }
    }

    /* (2) the common solution on each + face seen from its owner: the + neighbour's
     * minus trace, L2-projected onto the owner's face points when the degrees differ */
    for (int k = 0; k < Ne; ++k) {
        const int P = deg[k] + 1, NF = ipow(P, dim - 1);
        for (int a = 0; a < dim; ++a) {
            int kp = neighbour(m, k, a, +1);
            const int Pn = deg[kp] + 1;
            double T[OR_MAXP * OR_MAXP];
            if (Pn != P) proj1d(Pn, P, T);
            for (int v = 0; v < nv; ++v) {
                if (Pn == P) {
                    for (int f = 0; f < NF; ++f) PT(Qs, a, v, f, k) = PT(Tm, a, v, f, kp);
                } else {
                    face_map(dim, Pn, P, T, &PT(Tm, a, v, 0, kp), (size_t)Ne, &PT(Qs, a, v, 0, k), (size_t)Ne);
                }
            }
        }
    }

    /* (3) corrected gradient (correction at the + end only, as in the uniform scheme) */
    for (int k = 0; k < Ne; ++k) {
        const int P = deg[k] + 1, Np = ipow(P, dim);
        int ck[3];
        elem_coords(m, k, ck);
        for (int c = 0; c < dim; ++c) {
            double jac = 2.0 / m->h[c][ck[c]];
            for (int v = 0; v < nv; ++v)
                for (int i = 0; i < Np; ++i) {
                    int f, ic;
                    point_split(dim, P, c, i, &f, &ic);
                    double s = 0.0;
                    for (int j = 0; j < P; ++j)
                        s += o[P].D[ic][j] * PQ(dq, v, line_point(dim, P, c, f, j), k);
                    s += (PT(Qs, c, v, f, k) - PT(Tp, c, v, f, k)) * o[P].gRd[ic];
                    PG(G, c, v, i, k) = jac * s;
                }
        }
    }

    /* (4) traces of every gradient component at the + end of each axis */
    for (int k = 0; k < Ne; ++k) {
        const int P = deg[k] + 1, NF = ipow(P, dim - 1);
        for (int a = 0; a < dim; ++a)
            for (int c = 0; c < dim; ++c)
                for (int v = 0; v < nv; ++v)
                    for (int f = 0; f < NF; ++f) {
                        double s = 0.0;
                        for (int j = 0; j < P; ++j)
                            s += o[P].bp[j] * PG(G, c, v, line_point(dim, P, a, f, j), k);
                        PGT(GTp, a, c, v, f, k) = s;
                    }
    }

    /* (5) pointwise flux deviation and (6) its traces along its own axis */
    for (int k = 0; k < Ne; ++k) {
        const int P = deg[k] + 1, Np = ipow(P, dim), NF = ipow(P, dim - 1);
        for (int i = 0; i < Np; ++i) {
            double q[5], grad[3][5];
            state_t s;
            for (int v = 0; v < nv; ++v) q[v] = PQ(dq, v, i, k);
            for (int c = 0; c < dim; ++c)
                for (int v = 0; v < nv; ++v) grad[c][v] = PG(G, c, v, i, k);
            primitives(dim, m->gamma, m->qinf, q, &s);
            for (int a = 0; a < dim; ++a) {
                double FI[5], FV[5];
                inviscid_dflux(dim, a, m->qinf, &s, FI);
                viscous_flux(dim, a, m->gamma, m->mu, m->Pr, &s, grad, FV);
                for (int v = 0; v < nv; ++v) PG(Fl, a, v, i, k) = FI[v] - FV[v];
            }
        }
        for (int a = 0; a < dim; ++a)
            for (int v = 0; v < nv; ++v)
                for (int f = 0; f < NF; ++f) {
                    double sm = 0.0, sp = 0.0;
                    for (int j = 0; j < P; ++j) {
                        double fl = PG(Fl, a, v, line_point(dim, P, a, f, j), k);
                        sm += o[P].bm[j] * fl;
                        sp += o[P].bp[j] * fl;
                    }
                    PT(FTm, a, v, f, k) = sm;
                    PT(FTp, a, v, f, k) = sp;
                }
    }

    /* (7) common flux on every face (the + face of k), at the mortar points
     * when the degrees differ; Fsp = on k's + face at k's points, Fsm = on the
     * + neighbour's - face at its points */
    for (int k = 0; k < Ne; ++k) {
        const int P = deg[k] + 1, NF = ipow(P, dim - 1);
        for (int a = 0; a < dim; ++a) {
            int kp = neighbour(m, k, a, +1);
            const int Pn = deg[kp] + 1;
            const int Pm = P > Pn ? P : Pn, NFm = ipow(Pm, dim - 1);
            double TL[OR_MAXP * OR_MAXP], TR_[OR_MAXP * OR_MAXP], TbL[OR_MAXP * OR_MAXP],
                TbR[OR_MAXP * OR_MAXP];
            if (P != Pm) { proj1d(P, Pm, TL); proj1d(Pm, P, TbL); }
            if (Pn != Pm) { proj1d(Pn, Pm, TR_); proj1d(Pm, Pn, TbR); }
            /* both traces and the owner's gradient trace at the mortar points */
            double qLm[5][OR_MAXP * OR_MAXP], qRm[5][OR_MAXP * OR_MAXP], gm[3][5][OR_MAXP * OR_MAXP];
            double Fm[5][OR_MAXP * OR_MAXP];
            for (int v = 0; v < nv; ++v) {
                if (P == Pm) {
                    for (int f = 0; f < NFm; ++f) qLm[v][f] = PT(Tp, a, v, f, k);
                    for (int c = 0; c < dim; ++c)
                        for (int f = 0; f < NFm; ++f) gm[c][v][f] = PGT(GTp, a, c, v, f, k);
                } else {
                    face_map(dim, P, Pm, TL, &PT(Tp, a, v, 0, k), (size_t)Ne, qLm[v], 1);
                    for (int c = 0; c < dim; ++c)
                        face_map(dim, P, Pm, TL, &PGT(GTp, a, c, v, 0, k), (size_t)Ne, gm[c][v], 1);
                }
                if (Pn == Pm) {
                    for (int f = 0; f < NFm; ++f) qRm[v][f] = PT(Tm, a, v, f, kp);
                } else {
                    face_map(dim, Pn, Pm, TR_, &PT(Tm, a, v, 0, kp), (size_t)Ne, qRm[v], 1);
                }
            }
            for (int f = 0; f < NFm; ++f) {
                double qL[5], qR[5], Fr[5], FV[5], grad[3][5];
                state_t sL;
                for (int v = 0; v < nv; ++v) {
                    qL[v] = qLm[v][f];
                    qR[v] = qRm[v][f];
                }
                for (int c = 0; c < dim; ++c)
                    for (int v = 0; v < nv; ++v) grad[c][v] = gm[c][v][f];
                roe_dflux(dim, a, m->gamma, m->qinf, qL, qR, Fr);
                primitives(dim, m->gamma, m->qinf, qL, &sL);
                viscous_flux(dim, a, m->gamma, m->mu, m->Pr, &sL, grad, FV);
                for (int v = 0; v < nv; ++v) Fm[v][f] = Fr[v] - (FV[v] + m->tau * (qR[v] - qL[v]));
            }
            for (int v = 0; v < nv; ++v) {
                if (P == Pm) {
                    for (int f = 0; f < NF; ++f) PT(Fsp, a, v, f, k) = Fm[v][f];
                } else {
                    face_map(dim, Pm, P, TbL, Fm[v], 1, &PT(Fsp, a, v, 0, k), (size_t)Ne);
                }
                if (Pn == Pm) {
                    for (int f = 0; f < ipow(Pn, dim - 1); ++f) PT(Fsm, a, v, f, kp) = Fm[v][f];
                } else {
                    face_map(dim, Pm, Pn, TbR, Fm[v], 1, &PT(Fsm, a, v, 0, kp), (size_t)Ne);
                }
            }
        }
    }

    /* (8) R = -sum_a (2/h_a) [D f_a + (F*_- - f^-) g_L' + (F*_+ - f^+) g_R'] */
    for (int k = 0; k < Ne; ++k) {
        const int P = deg[k] + 1, Np = ipow(P, dim);
        int ck[3];
        elem_coords(m, k, ck);
        for (int v = 0; v < nv; ++v) {
            for (int i = 0; i < Np; ++i) {
                double acc = 0.0;
                for (int a = 0; a < dim; ++a) {
                    int f, ia;
                    point_split(dim, P, a, i, &f, &ia);
                    double s = 0.0;
                    for (int j = 0; j < P; ++j)
                        s += o[P].D[ia][j] * PG(Fl, a, v, line_point(dim, P, a, f, j), k);
                    s += (PT(Fsm, a, v, f, k) - PT(FTm, a, v, f, k)) * o[P].gLd[ia];
                    s += (PT(Fsp, a, v, f, k) - PT(FTp, a, v, f, k)) * o[P].gRd[ia];
                    acc += (2.0 / m->h[a][ck[a]]) * s;
                }
                PQ(r, v, i, k) = -acc;
            }
            for (int i = Np; i < NpM; ++i) PQ(r, v, i, k) = 0.0;
        }
    }
#undef PQ
#undef PT
#undef PG
#undef PGT
    free(Tm); free(Tp); free(Qs); free(G); free(GTp); free(Fl); free(FTm); free(FTp); free(Fsp); free(Fsm);
    return 0;
}

/* EJ blocks on a mixed-degree mesh, as or_ej_blocks (same colouring, step
 * and one-sided difference) with or_residual_pa.  Blocks are n_b = nvar
 * m->P^dim square in the padded numbering v m->P^dim + i; the rows and
 * columns of element k's unused points hold the identity. */
int or_ej_blocks_pa(const or_mesh *m, const int *deg, const double *dq, const double *r0, double sigma, double *B)
{
    const int dim = m->dim, nv = dim + 2;
    const int Ne = mesh_ne(m), Np = ipow(m->P, dim), nb = nv * Np;
    for (int a = 0; a < dim; ++a)
        if (m->n[a] % 2 != 0) return -1;
    size_t N = (size_t)nv * Np * Ne;
    double *qp = malloc(sizeof(double) * N);
    double *rp = malloc(sizeof(double) * N);
    double *hk = malloc(sizeof(double) * Ne);
    int *col = malloc(sizeof(int) * Ne);
    if (!qp || !rp || !hk || !col) { free(qp); free(rp); free(hk); free(col); return -2; }
    for (int k = 0; k < Ne; ++k) {
        int c[3];
        elem_coords(m, k, c);
        col[k] = (c[0] & 1) | ((c[1] & 1) << 1) | ((c[2] & 1) << 2);
    }
    for (int k = 0; k < Ne; ++k) {
        double *Bk = B + (size_t)k * nb * nb;
        memset(Bk, 0, sizeof(double) * nb * nb);
        for (int j = 0; j < nb; ++j) Bk[(size_t)j * nb + j] = 1.0;
    }
    int ncol = 1 << dim;
    for (int colour = 0; colour < ncol; ++colour)
        for (int j = 0; j < nb; ++j) {
            int jv = j / Np, ji = j % Np;
            int any = 0;
            memcpy(qp, dq, sizeof(double) * N);
            for (int k = 0; k < Ne; ++k) {
                hk[k] = 0.0;
                if (col[k] != colour || ji >= ipow(deg[k] + 1, dim)) continue;
                size_t idx = ((size_t)jv * Np + ji) * Ne + k;
                double hj = 1e-7 * fmax(1.0, fabs(m->qinf[jv] + dq[idx]));
                qp[idx] = dq[idx] + hj;
                hk[k] = qp[idx] - dq[idx];
                any = 1;
            }
            if (!any) continue;
            int rc = or_residual_pa(m, deg, qp, rp);
            if (rc) { free(qp); free(rp); free(hk); free(col); return rc; }
            for (int k = 0; k < Ne; ++k) {
                if (hk[k] == 0.0) continue;
                const int Npk = ipow(deg[k] + 1, dim);
                double *Bk = B + (size_t)k * nb * nb;
                for (int row = 0; row < nb; ++row) {
                    if (row % Np >= Npk) continue;
                    size_t idx = (size_t)row * Ne + k;
                    Bk[(size_t)row * nb + j] = (row == j ? sigma : 0.0) - (rp[idx] - r0[idx]) / hk[k];
                }
            }
        }
    free(qp); free(rp); free(hk); free(col);
    return 0;
}
