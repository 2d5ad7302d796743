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

// 1D SIP element matrices, reference cell [0,1], penalty Cr (times 1/h on
// the physical cell, so every entry scales as 1/h).
void build_line_matrix(int n, const double* W, const double* D, const double* L0, const double* L1,
                   const double* dL0, const double* dL1, double Cr, Line1D& m) {
    std::memset(&m, 0, sizeof(m));
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double a = 0.0;
            for (int q = 0; q < n; ++q) a += W[q] * D[q * n + i] * D[q * n + j];
            const double f0 = 0.5 * dL0[j] * L0[i] + 0.5 * L0[j] * dL0[i] + Cr * L0[i] * L0[j];
            const double f1 = -0.5 * dL1[j] * L1[i] - 0.5 * L1[j] * dL1[i] + Cr * L1[i] * L1[j];
            m.F0[i * n + j] = f0;
            m.F1[i * n + j] = f1;
            m.A[i * n + j] = a + f0 + f1;
            m.Lm[i * n + j] = 0.5 * dL1[j] * L0[i] - 0.5 * L1[j] * dL0[i] - Cr * L0[i] * L1[j];
            m.Rm[i * n + j] = -0.5 * dL0[j] * L1[i] + 0.5 * L0[j] * dL1[i] - Cr * L1[i] * L0[j];
            m.WD[i * n + j] = W[i] * D[i * n + j];   // row m = i, column = test function j
        }
}

double lagrange_value(const double* z, int n, int j, double x) { return lagrange(z, n, j, x); }

// Pressure-type tables of one multigrid level with np Gauss nodes per
// direction: rule, derivative matrix, end values and derivatives, the 1D SIP
// element matrices with the reference penalty np^2 pen_p.
void level_tables(int np, double pen_p, Tables& t, Line1D& line, double& cr) {
    std::memset(&t, 0, sizeof(t));
    gauss_legendre(np, t.xp, t.Wp);
    for (int i = 0; i < np; ++i)
        for (int j = 0; j < np; ++j) t.Dp[i * np + j] = lagrange_d(t.xp, np, j, t.xp[i]);
    for (int j = 0; j < np; ++j) {
        t.L0p[j] = lagrange(t.xp, np, j, 0.0);
        t.L1p[j] = lagrange(t.xp, np, j, 1.0);
        t.dL0p[j] = lagrange_d(t.xp, np, j, 0.0);
        t.dL1p[j] = lagrange_d(t.xp, np, j, 1.0);
    }
    cr = (double)np * np * pen_p;
    build_line_matrix(np, t.Wp, t.Dp, t.L0p, t.L1p, t.dL0p, t.dL1p, cr, line);
}

void build_line_operators(tbdg_ctx* c) {
    const Tables& t = c->tab;
    c->cr_u = (c->k + 1.0) * (c->k + 1.0) * c->pen_u;
    c->cr_p = (double)c->k * c->k * c->pen_p;
    build_line_matrix(c->n, t.Wu, t.Du, t.L0u, t.L1u, t.dL0u, t.dL1u,
                  (c->k + 1.0) * (c->k + 1.0) * c->pen_u, c->line_u);
    build_line_matrix(c->np, t.Wp, t.Dp, t.L0p, t.L1p, t.dL0p, t.dL1p,
                  (double)c->k * c->k * c->pen_p, c->line_p);
    for (int a = 0; a < 3; ++a) {
        c->lgeom.periodic[a] = c->periodic_flags[a];
        c->lgeom.inv_nc[a] = 1.0 / c->geom.nc[a];
        c->lgeom.sadv[a] = c->geom.vol / c->geom.h[a];
        c->lgeom.sdiff[a] = c->geom.vol / (c->geom.h[a] * c->geom.h[a]);
    }
    c->lgeom.wall = -1.0;   // pressure forms: natural condition at walls
}

}  // namespace trbdg

double tbdg_ctx::alpha(int s) const {
    if (std::isinf(c)) return 0.0;
    return 1.0 / (c * c * beta[s] * beta[s] * dt * dt);
}

namespace trbdg {

// Vertices of the Q1-mapped 2D mesh: the Cartesian grid point (x, y) moves
// by amp sin(2 pi x) sin(2 pi y) in both coordinates (the distortion of the
// Kovasznay workload; it vanishes on box edges at multiples of 1/2).  Every
// cell keeps its own four vertices (cells at a periodic wrap keep their
// unwrapped shape).  gr holds |Gamma| / |K| per face (a, s): the edge length
// over the cell area, both exact for the bilinear map.
void build_mapped_geometry(const tbdg_ctx* c, double amp, std::vector<double>& vtx,
                           std::vector<double>& gr) {
    const int n0 = c->geom.nc[0], n1 = c->geom.nc[1];
    const double pi2 = 2.0 * std::acos(-1.0);
    auto vert = [&](int i, int j, double* out) {
        const double x = c->geom.lo[0] + i * c->geom.h[0];
        const double y = c->geom.lo[1] + j * c->geom.h[1];
        const double d = amp * std::sin(pi2 * x) * std::sin(pi2 * y);
        out[0] = x + d;
        out[1] = y + d;
    };
    vtx.assign((size_t)c->Nc * 8, 0.0);
    gr.assign((size_t)c->Nc * 4, 0.0);
    for (int j = 0; j < n1; ++j)
        for (int i = 0; i < n0; ++i) {
            const size_t cell = (size_t)i + (size_t)n0 * j;
            double* X = &vtx[cell * 8];
            for (int v = 0; v < 4; ++v) vert(i + (v & 1), j + (v >> 1), X + 2 * v);
            // area of the quadrilateral 0-1-3-2: half the cross product of the diagonals
            const double d1x = X[6] - X[0], d1y = X[7] - X[1];
            const double d2x = X[4] - X[2], d2y = X[5] - X[3];
            const double area = 0.5 * std::fabs(d1x * d2y - d1y * d2x);
            auto len = [&](int p, int q) { return std::hypot(X[2 * q] - X[2 * p], X[2 * q + 1] - X[2 * p + 1]); };
            gr[cell * 4 + 0] = len(0, 2) / area;   // xi0 = 0
            gr[cell * 4 + 1] = len(1, 3) / area;   // xi0 = 1
            gr[cell * 4 + 2] = len(0, 1) / area;   // xi1 = 0
            gr[cell * 4 + 3] = len(2, 3) / area;   // xi1 = 1
        }
}

}  // namespace trbdg
