// Adaptive 2D quadrilateral meshes with hanging nodes: the device-side view
// shared by the host forest (amr.cpp) and the kernels (amr.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace trbdg {
namespace amr {

constexpr int MAXN = 8;   // nodes per direction (velocity degree <= 7)

// Face neighbour kinds of one cell face (meta & 15); a coarser neighbour
// carries the half of its face this cell touches in meta >> 4.
enum : int { FACE_BOUNDARY = 0, FACE_SAME = 1, FACE_COARSER = 2, FACE_FINER = 3 };

// 1D tables of one nodal basis (n Gauss-Legendre nodes on [0,1]).
struct Tab1 {
    int n;
    double z[MAXN], W[MAXN];
    double D[MAXN * MAXN];        // D[m n + j] = l_j'(z_m)
    double S[MAXN * MAXN];        // S[i n + j] = sum_m W_m D[m][i] D[m][j]
    double L[2][MAXN];            // l_j(0), l_j(1)
    double dL[2][MAXN];           // l_j'(0), l_j'(1)
    double T[2][MAXN * MAXN];     // T[h][q n + m] = l_m((h + z_q) / 2)
};

// Pressure basis (np = n - 1 nodes) at the velocity Gauss points.
struct MixTab {
    int n, np;
    double I[MAXN * MAXN];        // I[q np + m] = l^p_m(z_q)
    double DI[MAXN * MAXN];       // DI[q np + m] = (l^p_m)'(z_q)
    double Ih[2][MAXN * MAXN];    // Ih[h][q np + m] = l^p_m((h + z_q) / 2)
    double Lp[2][MAXN];           // l^p_m(0), l^p_m(1)
};

// Cells in the order of the forest; face f = 2 a + s (direction a, side s).
struct Geo {
    const int* level;     // [Nc]
    const int* meta;      // [Nc][4]
    const int* nbr;       // [Nc][4][2]: the neighbour, or the two finer ones
    const int* bface;     // [Nc][4]: boundary face number (cell, face order), or -1
    int Nc;
    double H[2];          // base cell size per direction
    double csig;          // pressure: k^2 times the penalty multiplier
    double csig_u;        // velocity: (k+1)^2 times the penalty multiplier
};

// Source of every new cell in a transfer: kind 0 copy of src[0], kind 1
// child (position bx + 2 by) of src[0], kind 2 parent of src[0..3] (children
// (0,0), (1,0), (0,1), (1,1)).
struct XferMap {
    const int* kind;      // [Nnew]: kind | (child position << 4)
    const int* src;       // [Nnew][4]
    int Nnew;
};

// The fused CG direction of the pressure operator: the operand is
// p_new = z + beta p_old, beta = r.z / *rz_old (0 and p_old unread when
// rz_old is null), written to pnew (which must not alias z or pold).  r.z
// is *rz_new, or, when rz_part is not null, the sum of its rz_G partials,
// which block 0 then stores in rz_store (if not null; rz_store must differ
// from rz_old).
struct CgDir {
    const double* pold;
    double* pnew;
    const double* rz_new;
    const double* rz_part;
    int rz_G;
    const double* rz_old;
    double* rz_store;
};

// The CG update fused into the preconditioner: x += al p, r -= al q,
// al = *rz / p.q with p.q the scalar *pq or, when pq_part is not null, the
// sum of its pq_G partials
struct CgUpdate {
    const double* rz;
    const double* pq;
    const double* pq_part;
    int pq_G;
    const double* p;
    const double* q;
    double* x;
};

// part (may be null): per-block partial sums of p . y, amr_pressure_blocks
// of them
void launch_amr_pressure(hipStream_t st, const Geo& g, const Tab1& t, double alpha, const double* p,
                         double* y, bool diag, double* part = nullptr);
int amr_pressure_blocks(const Geo& g, const Tab1& t);
// mode 0 apply, 1 diagonal, 2 the cell-local part (exterior traces zero)
void launch_amr_pressure_mode(hipStream_t st, const Geo& g, const Tab1& t, double alpha,
                              const double* p, double* y, int mode, double* part);
// q = H p_new with p_new = z + beta p_old formed and stored on the way, and
// the per-block partials of p_new . q in part
void launch_amr_pressure_dir(hipStream_t st, const Geo& g, const Tab1& t, double alpha, const double* z,
                             const CgDir& dir, double* q, double* part);
void launch_amr_pressure_any(hipStream_t st, const Geo& g, const Tab1& t, double alpha, const double* p,
                             double* y, int mode, double* part, const CgDir& dir);
// cell-block Jacobi of the pressure operator (blocks of 1, 4, 9 or 16 nodes):
// build FP32 block inverses (u, y: pressure-size scratch, B: FP64 blocks),
// apply z = B^{-1} r with block partials of r.z and r.r (returns the grid)
bool amr_block_ok(int nb);
void launch_amr_block_build(hipStream_t st, const Geo& g, const Tab1& t, double alpha, double* u,
                            double* y, double* B, float* Binv);
int launch_amr_block_apply(hipStream_t st, int64_t nc, int nb, const float* Binv, const double* r,
                           double* z, double* part);
// the grid of the block preconditioner (cells / (256 / nb) blocks)
int amr_block_grid(int64_t nc, int nb);
// the same after the CG update of x and r (returns the grid)
int launch_amr_block_xr(hipStream_t st, int64_t nc, int nb, const float* Binv, const CgUpdate& xr,
                        double* r, double* z, double* part);
// the update u of x and r, then z = r / d, with block partials of r.z and
// r.r in part[0..G), part[G..2G)
void launch_amr_cg_step(hipStream_t st, int64_t n, const CgUpdate& u, const double* d, double* r,
                        double* z, double* part, int G);
// out0 = sum of part[0..G), out1 = sum of part[G..2G) when rows == 2
void launch_amr_finish(hipStream_t st, const double* part, int G, int rows, double* out0, double* out1);
// y_c = mc M u_c + tnu A u_c + th C(w) u_c, c = 0, 1; uD: wall data at the
// velocity Gauss points of the boundary faces (face number bface, n points)
void launch_amr_momentum(hipStream_t st, const Geo& g, const Tab1& t, double mc, double tnu, double th,
                         const double* w, const double* u, const double* uD, double* y);
// Momentum right-hand side pieces, both components:
//   y_c (+)= mcoef M uprev_c + cl L0 ue_c + ca A0_we(ue)_c + cg (Gw p)_c
//            + wall-data terms (thd, visc, wd, uD) of the stage functional
// L0, A0 the explicit diffusion and advection of eq. rhs1 over the whole
// skeleton, Gw the weak gradient; p, uD, wd may be null when unused.
struct ExplicitArgs {
    double mcoef, cl, ca, cg, thd, visc;
    const double *uprev, *ue, *we, *p, *wd, *uD;
    bool acc;
};
void launch_amr_explicit(hipStream_t st, const Geo& g, const Tab1& t, const MixTab& x,
                         const ExplicitArgs& e, double* y);
// b = alpha M^p p + fcoef D u (the Helmholtz right-hand side of a stage)
void launch_amr_rhs_p(hipStream_t st, const Geo& g, const Tab1& t, const MixTab& x, double alpha,
                      const double* p, double fcoef, const double* u, double* b);
// y = x + a M^{-1} P p (the nodal gradient of p at the velocity nodes)
void launch_amr_grad(hipStream_t st, const Geo& g, const Tab1& t, const MixTab& x, const double* xin,
                     double a, const double* p, double* y);
// diag(mc M + tnu A) in the velocity layout (both components)
void launch_amr_momentum_diag(hipStream_t st, const Geo& g, const Tab1& t, double mc, double tnu,
                              double* d);
void launch_amr_indicator(hipStream_t st, const Geo& g, const Tab1& t, const double* u, double* eta);
void launch_amr_transfer(hipStream_t st, const XferMap& m, const Tab1& t, int ncomp, const double* src,
                         double* dst);
// partial sums of a.b over G blocks into part, then the sum into *out
void launch_amr_dot(hipStream_t st, int64_t n, const double* a, const double* b, double* part, int G,
                    double* out);
// max |a - b| over G block partials in part, then into *out
void launch_amr_maxdiff(hipStream_t st, int64_t n, const double* a, const double* b, double* part, int G,
                       double* out);
void launch_amr_div(hipStream_t st, int64_t n, const double* r, const double* d, double* z);

}  // namespace amr
}  // namespace trbdg
