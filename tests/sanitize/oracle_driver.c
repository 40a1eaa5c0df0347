/* Drives every C entry point of the oracle (fr_oracle.c, compiled into the
 * same executable) on small 2D and 3D meshes, for the address and
 * undefined-behaviour sanitizer build in tests/test_oracle_sanitizers.py.
 * Exit status 0 and no sanitizer report: every access stayed in bounds. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "../../oracle/fr_oracle.c"

static double frand(unsigned *s)
{
    *s = *s * 1664525u + 1013904223u;
    return ((*s >> 8) / 16777216.0) - 0.5;
}

static int run(int dim, const int n[3], int P, unsigned seed)
{
    double hx[8], hy[8], hz[8];
    for (int i = 0; i < 8; ++i) {
        hx[i] = 0.1 + 0.01 * i;
        hy[i] = 0.2 - 0.01 * i;
        hz[i] = 0.15;
    }
    or_mesh m;
    m.dim = dim;
    m.P = P;
    m.n[0] = n[0];
    m.n[1] = n[1];
    m.n[2] = dim == 3 ? n[2] : 1;
    m.h[0] = hx;
    m.h[1] = hy;
    m.h[2] = hz;
    m.gamma = 1.4;
    m.mu = 1e-2;
    m.Pr = 0.72;
    m.tau = 0.1;
    const double pinf = 1.0 / (1.4 * 0.3 * 0.3);
    m.qinf[0] = 1.0;
    m.qinf[1] = 0.8;
    m.qinf[2] = 0.6;
    m.qinf[3] = dim == 3 ? 0.0 : pinf / 0.4 + 0.5;
    m.qinf[4] = pinf / 0.4 + 0.5;
    const int nv = dim + 2;
    int Np = 1;
    for (int a = 0; a < dim; ++a) Np *= P;
    const int Ne = m.n[0] * m.n[1] * m.n[2];
    const int nb = nv * Np;
    const size_t N = (size_t)nv * Np * Ne;
    double *dq = malloc(sizeof(double) * N), *r = malloc(sizeof(double) * N), *y = malloc(sizeof(double) * N);
    double *B = malloc(sizeof(double) * (size_t)Ne * nb * nb);
    int32_t *piv = malloc(sizeof(int32_t) * (size_t)Ne * nb);
    for (size_t i = 0; i < N; ++i) dq[i] = 0.02 * frand(&seed);
    int rc = or_residual(&m, dq, r);
    if (!rc) rc = or_ej_blocks(&m, dq, r, 50.0, B);
    if (!rc) rc = or_lu_factor_batch(Ne, nb, B, piv);
    if (!rc) or_lu_solve_batch(Ne, nb, B, piv, r, y);
    double s = 0.0;
    for (size_t i = 0; i < N; ++i) s += y[i] * y[i];
    printf("dim %d P %d: rc %d, |y| %.6e\n", dim, P, rc, sqrt(s));
    free(dq);
    free(r);
    free(y);
    free(B);
    free(piv);
    return rc != 0 || !isfinite(s);
}

int main(void)
{
    int fail = 0;
    for (int P = 1; P <= 5; ++P) {
        double out[5 * 5 + 6 * 5], x[5], w[5];
        or_ops1d(P, out);
        or_gauss_legendre(P, x, w);
        for (int P1 = 1; P1 < P; ++P1) {
            double G[25], Pi[25];
            or_transfer1d(P, P1, G, Pi);
        }
    }
    const double qinf[5] = {1.0, 0.8, 0.6, 0.1, 30.0};
    const double dqL[5] = {0.01, -0.02, 0.03, 0.01, 0.2}, dqR[5] = {-0.01, 0.02, 0.01, -0.03, -0.1};
    double F[5], grad[15];
    for (int i = 0; i < 15; ++i) grad[i] = 0.1 * (i % 7) - 0.3;
    for (int dim = 2; dim <= 3; ++dim)
        for (int a = 0; a < dim; ++a) {
            or_inviscid_dflux(dim, a, 1.4, qinf, dqL, F);
            or_roe_dflux(dim, a, 1.4, qinf, dqL, dqR, F);
            or_viscous_flux(dim, a, 1.4, 1e-2, 0.72, qinf, dqL, grad, F);
        }
    const int n2[3] = {4, 4, 1}, n3[3] = {4, 2, 2};
    for (int P = 1; P <= 5; ++P) fail |= run(2, n2, P, 11u + P);
    for (int P = 1; P <= 4; ++P) fail |= run(3, n3, P, 23u + P);
    return fail;
}
