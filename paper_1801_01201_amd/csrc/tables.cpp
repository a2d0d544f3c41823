// SDC coefficient tables computed on the host in extended precision.
//
// Section 3.1 of the paper: Gauss-Lobatto nodes, the integration matrix Q
// (q_{m+1,j} = integral from t^0 to t^{m+1} of the Lagrange polynomial L_j,
// divided by dt), the LU-trick implicit weights Q~I = transpose of the upper
// factor U of transpose(Q~) = L U (Doolittle: L unit lower triangular), the
// cumulative backward-Euler weights used by MISDC, and the forward-Euler
// explicit weights Q~E.  Nodes are found by Newton's method on P'_M in long
// double; the integrals of the Lagrange basis are evaluated exactly with a
// Gauss-Legendre rule of sufficient degree, also in long double.
#include <cmath>

#include "misdc_impl.h"

namespace misdc {

namespace {

using ld = long double;

// Legendre P_n(x) and its derivative by the three-term recurrence.
void legendre(int n, ld x, ld& p, ld& dp) {
    ld p0 = 1, p1 = x;
    if (n == 0) { p = 1; dp = 0; return; }
    for (int k = 2; k <= n; ++k) {
        ld pk = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = pk;
    }
    p = p1;
    dp = n * (x * p1 - p0) / (x * x - 1);   // valid for |x| < 1
}

// Interior Lobatto points on (-1, 1): roots of P'_M, via Newton on P'_M
// with P''_M from the Legendre differential equation.
void lobatto_interior(int M, ld* out) {
    const ld pi = 3.14159265358979323846264338327950288L;
    for (int k = 1; k < M; ++k) {
        ld x = -std::cos(pi * k / M);
        for (int it = 0; it < 100; ++it) {
            ld p, dp;
            legendre(M, x, p, dp);
            // (1 - x^2) P'' = 2 x P' - M (M+1) P
            ld d2p = (2 * x * dp - M * (M + 1) * p) / (1 - x * x);
            ld dx = dp / d2p;
            x -= dx;
            if (std::fabs(dx) < 1e-30L) break;
        }
        out[k - 1] = x;
    }
}

// Gauss-Legendre nodes/weights on [-1, 1] (n points) by Newton's method.
void gauss_legendre(int n, ld* x, ld* w) {
    const ld pi = 3.14159265358979323846264338327950288L;
    for (int i = 0; i < n; ++i) {
        ld z = std::cos(pi * (i + 0.75L) / (n + 0.5L));
        ld p, dp;
        for (int it = 0; it < 100; ++it) {
            legendre(n, z, p, dp);
            ld dz = p / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-30L) break;
        }
        legendre(n, z, p, dp);
        x[i] = z;
        w[i] = 2 / ((1 - z * z) * dp * dp);
    }
}

ld lagrange(int j, int n, const ld* tau, ld t) {
    ld v = 1;
    for (int i = 0; i < n; ++i)
        if (i != j) v *= (t - tau[i]) / (tau[j] - tau[i]);
    return v;
}

// integral over [a, b] of L_j (degree n-1 polynomial), exact with ng >= n/2 points
ld integrate_lagrange(int j, int n, const ld* tau, ld a, ld b) {
    const int ng = 8;
    ld gx[ng], gw[ng];
    gauss_legendre(ng, gx, gw);
    ld s = 0;
    for (int i = 0; i < ng; ++i) {
        ld t = 0.5L * (a + b) + 0.5L * (b - a) * gx[i];
        s += gw[i] * lagrange(j, n, tau, t);
    }
    return 0.5L * (b - a) * s;
}

}  // namespace

int make_tables(int n_nodes, int qi_kind, int qe_mode, Tables& t) {
    if (n_nodes < 2 || n_nodes > MAX_NODES)
        return fail(MISDC_EINVAL, "n_nodes must be in [2, %d], got %d", MAX_NODES, n_nodes);
    if (qi_kind != MISDC_QI_LU && qi_kind != MISDC_QI_BE)
        return fail(MISDC_EINVAL, "unknown implicit weights kind %d", qi_kind);
    if (qe_mode != MISDC_QE_CUMULATIVE && qe_mode != MISDC_QE_LITERAL)
        return fail(MISDC_EINVAL, "unknown explicit weights mode %d", qe_mode);
    const int M = n_nodes - 1;
    ld tau[MAX_NODES + 1];
    ld inner[MAX_NODES];
    lobatto_interior(M, inner);
    tau[0] = 0;
    for (int k = 1; k < M; ++k) tau[k] = (inner[k - 1] + 1) / 2;
    tau[M] = 1;

    ld Q[MAX_NODES][MAX_NODES + 1], S[MAX_NODES][MAX_NODES + 1];
    for (int p = 1; p <= M; ++p)
        for (int j = 0; j <= M; ++j) {
            S[p - 1][j] = integrate_lagrange(j, M + 1, tau, tau[p - 1], tau[p]);
            Q[p - 1][j] = integrate_lagrange(j, M + 1, tau, 0, tau[p]);
        }
    // Doolittle LU of A = transpose(Q~), Q~[p][j] = Q[p][j+1]
    ld A[MAX_NODES][MAX_NODES], L[MAX_NODES][MAX_NODES] = {}, U[MAX_NODES][MAX_NODES] = {};
    for (int a = 0; a < M; ++a)
        for (int b = 0; b < M; ++b) A[a][b] = Q[b][a + 1];
    for (int i = 0; i < M; ++i) {
        L[i][i] = 1;
        for (int k = i; k < M; ++k) {
            ld s = A[i][k];
            for (int q = 0; q < i; ++q) s -= L[i][q] * U[q][k];
            U[i][k] = s;
        }
        for (int k = i + 1; k < M; ++k) {
            ld s = A[k][i];
            for (int q = 0; q < i; ++q) s -= L[k][q] * U[q][i];
            L[k][i] = s / U[i][i];
        }
    }
    t = Tables();
    t.M = M;
    for (int k = 0; k <= M; ++k) t.tau[k] = (double)tau[k];
    for (int p = 0; p < M; ++p) {
        for (int j = 0; j <= M; ++j) {
            t.Q[p][j] = (double)Q[p][j];
            t.S[p][j] = (double)S[p][j];
        }
        for (int j = 0; j < M; ++j) {
            // QI[p][j] = U^T[p][j] = U[j][p]
            if (qi_kind == MISDC_QI_LU)
                t.QI[p][j] = (j <= p) ? (double)U[j][p] : 0.0;
            else
                t.QI[p][j] = (j <= p) ? (double)(tau[j + 1] - tau[j]) : 0.0;
            double qe = 0.0;
            if (qe_mode == MISDC_QE_CUMULATIVE) {
                if (j < p) qe = (double)(tau[j + 2] - tau[j + 1]);
            } else {
                if (j == p - 1) qe = (double)(tau[p + 1] - tau[p]);
            }
            t.QE[p][j] = qe;
        }
    }
    return MISDC_OK;
}

}  // namespace misdc

extern "C" int misdc_sdc_tables(int n_nodes, int qi_kind, int qe_mode, double* tau, double* Q,
                                double* QI, double* QE, double* S) {
    misdc::Tables t;
    int rc = misdc::make_tables(n_nodes, qi_kind, qe_mode, t);
    if (rc) return rc;
    const int M = t.M;
    for (int k = 0; k <= M; ++k)
        if (tau) tau[k] = t.tau[k];
    for (int p = 0; p < M; ++p) {
        for (int j = 0; j <= M; ++j) {
            if (Q) Q[p * (M + 1) + j] = t.Q[p][j];
            if (S) S[p * (M + 1) + j] = t.S[p][j];
        }
        for (int j = 0; j < M; ++j) {
            if (QI) QI[p * M + j] = t.QI[p][j];
            if (QE) QE[p * M + j] = t.QE[p][j];
        }
    }
    return MISDC_OK;
}
