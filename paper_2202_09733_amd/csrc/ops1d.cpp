// Host construction of the 1D operators of the FR discretisation and of the
// p-multigrid transfers, for the GPU kernels.
//
//  - Gauss-Legendre points and weights (Newton on L_P, Chebyshev start).
//  - Lagrange differentiation and end interpolation in barycentric form.
//  - Huynh's DG-recovering correction functions: the left correction is the
//    right Radau polynomial ((-1)^p/2)(L_p - L_{p+1}), the right one its
//    mirror (1/2)(L_p + L_{p+1}); only their derivatives at the solution
//    points are needed.
//  - Restriction = L2 projection (M^{p1})^{-1} M^{p1 p0} (Sec. 3.1,
//    Eq. (projection)).  On Gauss-Legendre nodes it equals truncation of the
//    discrete Legendre expansion, which is how it is built here; the
//    prolongation (M^{p0})^{-1} M^{p0 p1} (Eq. (prolongation)) equals
//    Lagrange interpolation of the coarse polynomial because the coarse space
//    is nested in the fine one.
#include <cmath>

#include "internal.hpp"

namespace frpmg {

namespace {

// L_n(x) and (for |x| < 1) L_n'(x) from (1 - x^2) L_n' = n (L_{n-1} - x L_n).
void legendre_pair(int n, double x, double &Ln, double &dLn) {
    double pm1 = 1.0, p = x;
    if (n == 0) {
        Ln = 1.0;
        dLn = 0.0;
        return;
    }
    for (int k = 2; k <= n; ++k) {
        double pk = ((2 * k - 1) * x * p - (k - 1) * pm1) / k;
        pm1 = p;
        p = pk;
    }
    Ln = p;
    dLn = n * (pm1 - x * p) / (1.0 - x * x);
}

void bary_weights(int P, const double *x, double *w) {
    for (int j = 0; j < P; ++j) {
        double prod = 1.0;
        for (int m = 0; m < P; ++m)
            if (m != j) prod *= (x[j] - x[m]);
        w[j] = 1.0 / prod;
    }
}

// l_j(t) for all j by the barycentric formula (t must not be a node).
void bary_eval(int P, const double *x, const double *w, double t, double *out) {
    double den = 0.0;
    for (int m = 0; m < P; ++m) den += w[m] / (t - x[m]);
    for (int j = 0; j < P; ++j) out[j] = (w[j] / (t - x[j])) / den;
}

}  // namespace

void gauss_legendre(int P, double *x, double *w) {
    for (int i = 0; i < P; ++i) {
        // Chebyshev-Gauss start, ascending order
        double t = -std::cos(M_PI * (2.0 * i + 1.0) / (2.0 * P));
        for (int it = 0; it < 60; ++it) {
            double L, dL;
            legendre_pair(P, t, L, dL);
            double step = L / dL;
            t -= step;
            if (std::fabs(step) <= 1e-16) break;
        }
        double L, dL;
        legendre_pair(P, t, L, dL);
        x[i] = t;
        w[i] = 2.0 / ((1.0 - t * t) * dL * dL);
    }
}

void build_ops1d(int P, Ops1D &o) {
    o = Ops1D{};
    double x[kMaxP], w[kMaxP], bw[kMaxP];
    gauss_legendre(P, x, w);
    bary_weights(P, x, bw);
    for (int i = 0; i < P; ++i) {
        double diag = 0.0;
        for (int j = 0; j < P; ++j) {
            if (j == i) continue;
            o.D[i][j] = (bw[j] / bw[i]) / (x[i] - x[j]);
            diag -= o.D[i][j];
        }
        o.D[i][i] = diag;
    }
    bary_eval(P, x, bw, -1.0, o.bm);
    bary_eval(P, x, bw, 1.0, o.bp);
    const int p = P - 1;
    const double sgn = (p % 2 == 0) ? 1.0 : -1.0;
    for (int i = 0; i < P; ++i) {
        double Lp, dLp, Lq, dLq;
        legendre_pair(p, x[i], Lp, dLp);
        legendre_pair(p + 1, x[i], Lq, dLq);
        o.gLd[i] = 0.5 * sgn * (dLp - dLq);
        o.gRd[i] = 0.5 * (dLp + dLq);
    }
    // the + end value of the nodal interpolant of D q and of gRd
    o.cgp = 0.0;
    for (int j = 0; j < P; ++j) {
        double sdn = 0.0;
        for (int i = 0; i < P; ++i) sdn += o.bp[i] * o.D[i][j];
        o.dnp[j] = sdn;
        o.cgp += o.bp[j] * o.gRd[j];
    }
}

void build_transfer(int P0, int P1, Transfer1D &t) {
    t = Transfer1D{};
    t.P0 = P0;
    t.P1 = P1;
    double x0[kMaxP], w0[kMaxP], x1[kMaxP], w1[kMaxP], bw1[kMaxP];
    gauss_legendre(P0, x0, w0);
    gauss_legendre(P1, x1, w1);
    // Gamma[a][i] = sum_{m < P1} L_m(x1_a) (2m+1)/2 w0_i L_m(x0_i)
    for (int a = 0; a < P1; ++a)
        for (int i = 0; i < P0; ++i) {
            double s = 0.0;
            for (int m = 0; m < P1; ++m) {
                double La, dLa, Li, dLi;
                legendre_pair(m, x1[a], La, dLa);
                legendre_pair(m, x0[i], Li, dLi);
                s += La * (2.0 * m + 1.0) * 0.5 * w0[i] * Li;
            }
            t.G[a][i] = s;
        }
    // Pi[i][j] = l_j^{coarse}(x0_i)
    bary_weights(P1, x1, bw1);
    for (int i = 0; i < P0; ++i) {
        double row[kMaxP];
        bool hit = false;
        for (int j = 0; j < P1; ++j)
            if (x0[i] == x1[j]) {
                hit = true;
                for (int m = 0; m < P1; ++m) row[m] = (m == j) ? 1.0 : 0.0;
            }
        if (!hit) bary_eval(P1, x1, bw1, x0[i], row);
        for (int j = 0; j < P1; ++j) t.Pi[i][j] = row[j];
    }
}

void build_pa_tables(PaTables &t) {
    t = PaTables{};
    for (int P = 1; P <= kMaxP; ++P) build_ops1d(P, t.ops[P]);
    // 1D L2 projection from the Pa-point to the Pb-point polynomial space:
    // truncation of the Legendre expansion for Pb < Pa, exact interpolation
    // for Pb > Pa, the identity for Pb = Pa
    for (int Pa = 1; Pa <= kMaxP; ++Pa)
        for (int Pb = 1; Pb <= kMaxP; ++Pb) {
            if (Pa == Pb) {
                for (int i = 0; i < Pa; ++i) t.proj[Pa][Pb][i][i] = 1.0;
            } else if (Pb < Pa) {
                Transfer1D tr;
                build_transfer(Pa, Pb, tr);
                for (int b = 0; b < Pb; ++b)
                    for (int a = 0; a < Pa; ++a) t.proj[Pa][Pb][b][a] = tr.G[b][a];
            } else {
                Transfer1D tr;
                build_transfer(Pb, Pa, tr);
                for (int b = 0; b < Pb; ++b)
                    for (int a = 0; a < Pa; ++a) t.proj[Pa][Pb][b][a] = tr.Pi[b][a];
            }
        }
    // Legendre coefficients of the P-point interpolant: c_n = (2n+1)/2 sum_i w_i L_n(x_i) s_i
    // (Gauss-Legendre with P points integrates L_n s, degree <= 2P - 2, exactly)
    for (int P = 1; P <= kMaxP; ++P) {
        double x[kMaxP], w[kMaxP];
        gauss_legendre(P, x, w);
        for (int n = 0; n < P; ++n)
            for (int i = 0; i < P; ++i) {
                double L, dL;
                legendre_pair(n, x[i], L, dL);
                t.modal[P][n][i] = (2.0 * n + 1.0) * 0.5 * w[i] * L;
            }
    }
}

}  // namespace frpmg
