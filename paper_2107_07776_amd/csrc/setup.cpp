// Context set-up: Gauss-Legendre rules by Newton iteration, Lagrange tables,
// geometry, penalties, workspaces.
#include <cmath>
#include <cstring>

#include "internal.hpp"

namespace trbdg {

// n-point Gauss-Legendre rule on [0,1]: roots of P_n by Newton iteration
// from the Chebyshev-like initial guesses cos(pi (i + 3/4) / (n + 1/2)).
void gauss_legendre(int n, double* x, double* w) {
    for (int i = 0; i < n; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int j = 2; j <= n; ++j) {
                const double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) p0 = 1.0;
            const double pn = (n == 1) ? z : p1;
            const double pm = (n == 1) ? 1.0 : p0;
            dp = n * (z * pn - pm) / (z * z - 1.0);
            const double dz = pn / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-17) break;
        }
        // recompute the derivative at the converged root
        double p0 = 1.0, p1 = z;
        for (int j = 2; j <= n; ++j) {
            const double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j;
            p0 = p1;
            p1 = p2;
        }
        const double pn = (n == 1) ? z : p1;
        const double pm = (n == 1) ? 1.0 : p0;
        dp = n * (z * pn - pm) / (z * z - 1.0);
        // ascending order on [0,1]
        x[n - 1 - i] = 0.5 * (z + 1.0);
        w[n - 1 - i] = 1.0 / ((1.0 - z * z) * dp * dp);   // 2/((1-z^2)P'^2) halved
    }
}

namespace {

double lagrange(const double* z, int n, int j, double x) {
    double v = 1.0;
    for (int m = 0; m < n; ++m)
        if (m != j) v *= (x - z[m]) / (z[j] - z[m]);
    return v;
}

double lagrange_d(const double* z, int n, int j, double x) {
    double s = 0.0;
    for (int m = 0; m < n; ++m) {
        if (m == j) continue;
        double t = 1.0 / (z[j] - z[m]);
        for (int q = 0; q < n; ++q)
            if (q != j && q != m) t *= (x - z[q]) / (z[j] - z[q]);
        s += t;
    }
    return s;
}

}  // namespace

void build_tables(tbdg_ctx* c) {
    Tables& t = c->tab;
    std::memset(&t, 0, sizeof(t));
    const int n = c->n, np = c->np;
    gauss_legendre(n, t.xu, t.Wu);
    gauss_legendre(np, t.xp, t.Wp);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) t.Du[i * n + j] = lagrange_d(t.xu, n, j, t.xu[i]);
    for (int j = 0; j < n; ++j) {
        t.L0u[j] = lagrange(t.xu, n, j, 0.0);
        t.L1u[j] = lagrange(t.xu, n, j, 1.0);
        t.dL0u[j] = lagrange_d(t.xu, n, j, 0.0);
        t.dL1u[j] = lagrange_d(t.xu, n, j, 1.0);
    }
    for (int i = 0; i < np; ++i)
        for (int j = 0; j < np; ++j) t.Dp[i * np + j] = lagrange_d(t.xp, np, j, t.xp[i]);
    for (int j = 0; j < np; ++j) {
        t.L0p[j] = lagrange(t.xp, np, j, 0.0);
        t.L1p[j] = lagrange(t.xp, np, j, 1.0);
        t.dL0p[j] = lagrange_d(t.xp, np, j, 0.0);
        t.dL1p[j] = lagrange_d(t.xp, np, j, 1.0);
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < np; ++j) {
            t.Ip[i * NMAX + j] = lagrange(t.xp, np, j, t.xu[i]);
            t.Dpu[i * NMAX + j] = lagrange_d(t.xp, np, j, t.xu[i]);
        }
}

}  // namespace trbdg

double tbdg_ctx::alpha(int s) const {
    if (std::isinf(c)) return 0.0;
    return 1.0 / (c * c * beta[s] * beta[s] * dt * dt);
}
