// Internal definitions shared by the host and device sources of libtrbdg.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/trbdg.h"

namespace trbdg {

constexpr int NMAX = 6;  // largest 1D node count (velocity degree 5)

// 1D tables on the reference interval [0,1].  Velocity: n Gauss nodes;
// pressure: np Gauss nodes.  D[i*N + j] = l_j'(x_i) (derivative of basis j at
// node i), L0/L1 = l_j(0)/l_j(1), dL0/dL1 = l_j'(0)/l_j'(1).  Mixed tables
// give the pressure basis at the velocity nodes: Ip[i*NMAX + j] = psi_j(xu_i),
// Dp[i*NMAX + j] = psi_j'(xu_i).  Passed by value as a kernel argument.
struct Tables {
    double Du[NMAX * NMAX];
    double Wu[NMAX], L0u[NMAX], L1u[NMAX], dL0u[NMAX], dL1u[NMAX];
    double Dp[NMAX * NMAX];
    double Wp[NMAX], L0p[NMAX], L1p[NMAX], dL0p[NMAX], dL1p[NMAX];
    double Ip[NMAX * NMAX], Dpu[NMAX * NMAX];
    double xu[NMAX], xp[NMAX];
};

// Uniform Cartesian box geometry (affine cells).
struct Geom {
    int nc[3];      // cells per direction (1 for unused directions)
    double h[3];    // cell size per direction
    double lo[3];
    double vol;     // |K|
};

// Element matrices of the one-dimensional SIP form on a reference cell of
// unit length (row i = test function, column j = trial function, stride n):
// A = cell stiffness + self terms of both end faces; F0/F1 = self terms of
// the left/right end face (subtracted where that face is a boundary);
// Lm/Rm = coupling to the left/right neighbour's basis.
// WD[m*n + i] = W_m l_i'(x_m) (volume advection weights).
struct Line1D {
    double A[NMAX * NMAX], F0[NMAX * NMAX], F1[NMAX * NMAX], Lm[NMAX * NMAX], Rm[NMAX * NMAX];
    double WD[NMAX * NMAX];
};

// Per-direction scale factors of the line operators on the affine box:
// sdiff[a] = |K| / h_a^2 (SIP), sadv[a] = |K| / h_a (advection).
// wall: the SIP form of a scalar field at a non-periodic end (no neighbour)
// takes the traces of the own cell's mirror image, even for the natural
// condition (-1: the pressure's homogeneous Neumann, no face terms) or odd
// for a homogeneous Dirichlet condition (+1: the velocity's boundary terms
// with the doubled penalty); read by the pressure-type line kernels only.
struct LineGeom {
    int periodic[3];
    double sdiff[3], sadv[3];
    double inv_nc[3];   // 1 / cells per direction (fast index division)
    double wall;
};

struct Error : std::runtime_error {
    tbdg_status status;
    Error(tbdg_status s, const std::string& m) : std::runtime_error(m), status(s) {}
};

#define TBDG_HIP(call)                                                          \
    do {                                                                        \
        hipError_t e_ = (call);                                                 \
        if (e_ != hipSuccess)                                                   \
            throw ::trbdg::Error(TBDG_EDEVICE, std::string(#call) + ": " +      \
                                 hipGetErrorString(e_));                        \
    } while (0)

// Event-bracketed timing of the operator kernels (measurement hook).
struct KTimer {
    bool on = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending[2];
    std::vector<hipEvent_t> pool;
    double total_ms[2] = {0.0, 0.0};
    int64_t count[2] = {0, 0};
    double bytes[2] = {0.0, 0.0};   // algorithmic bytes of the timed launches
};

// Dirichlet velocity data on the boundary faces of the box (the faces normal
// to non-periodic directions).  Face points are the tangential Gauss nodes of
// the velocity rule; face (a, side) holds one block per boundary cell, the
// cells in lexicographic order of their remaining coordinates, the points in
// the order of the line index of the operator kernels (lower direction
// fastest).
struct Bnd {
    const double* uD;       // [points][dim] at the stage time (zeros until set)
    int64_t off[3][2];      // first point of face (a, side); -1 for periodic directions
};

// Optional work fused into the momentum operator kernel for GMRES.  With
// invd set the operand is gsc[0] * invd (per scalar node) * u, the Jacobi-
// preconditioned Krylov vector, and the output is shifted:
// y = A (gsc[0] invd u) - shift gsc[0] u.  With ndot > 0 every block also
// writes the partial sums of y . V_i (i < ndot, stride ldv) and y . y to
// part[i * gridDim.x + block], i = 0 .. ndot.
struct MomFuse {
    const double* invd;
    const double* gsc;
    double shift;
    const double* V;
    int64_t ldv;
    int ndot;
    double* part;
    const double* shv;   // without invd: the shift is - shift gsc[0] shv (the Krylov vector)
    const double* rb = nullptr;   // residual mode: y = rb - (operator result)
};
constexpr int MOM_FUSE_MAX_DOTS = 8;

// Q1-mapped 2D mesh (device view): vertex coordinates per cell, vertex
// v = vx + 2 vy at vtx[(cell * 4 + v) * 2 + {0, 1}]; gr[cell * 4 + 2a + s] =
// |Gamma| / |K| of face (a, s); periodic flags and boundary-point offsets as
// on the affine box; uD the Dirichlet data of the stage.
struct MapMesh {
    const double* vtx;
    const double* gr;
    int nc[2];
    int per[2];
    int64_t off[2][2];
    const double* uD;
};

// Point index of the face point `tt` of boundary face (a, side) of `cell`.
__host__ __device__ inline int64_t bnd_point(const Bnd& b, const Geom& g, int64_t cell, int a,
                                             int side, int tt, int nf) {
    const int64_t c0 = cell % g.nc[0], c1 = (cell / g.nc[0]) % g.nc[1],
                  c2 = cell / ((int64_t)g.nc[0] * g.nc[1]);
    const int64_t tc = a == 0 ? c1 + (int64_t)g.nc[1] * c2
                     : (a == 1 ? c0 + (int64_t)g.nc[0] * c2 : c0 + (int64_t)g.nc[0] * c1);
    return b.off[a][side] + tc * nf + tt;
}

// ---- multigrid hierarchies (pressure; one velocity component) --------------------
constexpr int MG_MAXDEG = 16;     // largest Chebyshev degree
// smoother step kinds of the fused level kernel
enum { MG_PRE1 = 0, MG_STEP = 1, MG_LAST = 2, MG_RES = 3, MG_ZFIN = 4 };
constexpr int MG_MAXLEVELS = 16;

// FP32 1D tables of one level (row i = test function, column j = trial):
// A = SIP element matrix with both end-face self terms, L0/L1/dL0/dL1 = basis
// values/derivatives at the cell ends, W = Gauss weights; Cr = reference
// penalty; cm[s] = alpha_s |K| per stage; sdiff[a] = |K| / h_a^2; wall =
// LineGeom::wall.
struct LevelTabF {
    float A[NMAX * NMAX];
    float L0[NMAX], L1[NMAX], dL0[NMAX], dL1[NMAX], W[NMAX];
    float Cr;
    float wall;
    float cm[3];
    float sdiff[3];
};

// 1D transfer matrices to the next coarser level: T[b][i][j] = coarse Q1
// basis j at fine node i (b: child offset for an h-transfer, 0 for p).
struct TransferTab {
    float T[2][NMAX][2];
};

struct MGLevel {
    int np = 0;                 // nodes per direction (degree + 1)
    int64_t Nc = 0, N = 0;      // cells, DoFs
    Geom geom{};
    LineGeom lgeom{};
    Line1D line{};              // FP64 element matrices (setup, eigenvalue estimate)
    Tables tab{};               // FP64 pressure tables (only the *p entries are used)
    double cr = 0.0;
    LevelTabF tf{};
    int transfer = 0;           // to the next coarser level: 1 = p, 2 = h, 0 = coarsest
    TransferTab tt{};
    float *b = nullptr, *x = nullptr, *r = nullptr, *d[2] = {nullptr, nullptr};
    uint16_t *hb = nullptr, *hx = nullptr, *hr = nullptr, *hd[2] = {nullptr, nullptr};  // bf16 (level 0)
    float* invd[3] = {nullptr, nullptr, nullptr};
    double lam[3] = {0.0, 0.0, 0.0};      // eigenvalue estimate per stage
    double theta[3] = {0.0, 0.0, 0.0};
    double c1[3][MG_MAXDEG] = {}, c2[3][MG_MAXDEG] = {};
};

// The operator of every level is H_l = alpha_s M_l + K_l (K the SIP form of
// the level's degree with penalty factor pen, walls as in LineGeom::wall).
// Pressure: level 0 is the pressure space, alpha_s of the Helmholtz
// equation, natural walls.  Velocity (field 1): level 0 is the space of one
// velocity component, alpha_s = m_s / (theta_s nu) and Dirichlet walls, so
// that theta_s nu H_0 is the symmetric part (mass and diffusion) of the
// stage-s momentum operator on each component.
// The coarse end of a V-cycle run by one workgroup: the Q1 levels from some
// level below level 0 down to the coarsest, every vector resident in LDS
// (x, r, b, two directions and the inverse diagonal: 6 FP32 vectors per
// level), the same smoother,
// transfers and dense FP64 coarse solve as the level-by-level launches.
// Filled per stage by the host; passed by value.
constexpr int FUSE_MAXLV = 8;
constexpr int FUSE_THREADS = 1024;
struct FusedLv {
    int nc[3];
    int Nc, N, off;             // cells, DoFs, float offset of x (r, b, d0, d1, invd follow)
    float sdiff[3], cm, c2res;  // cm = alpha_s |K|; c2res = 1 / theta_s (residual step)
    float c1[MG_MAXDEG], c2[MG_MAXDEG];
    const float* invd;          // stage-s inverse diagonal (global)
};
struct FusedCycle {
    int nlev, degree;
    int periodic[3];
    float A[4], L0[2], L1[2], dL0[2], dL1[2], W[2], Cr, wall;
    TransferTab tt;             // h-transfer (the same for every pair of Q1 levels)
    const double* ainv;         // coarsest level's inverse (row-major, FP64)
    const float* b_top;         // right-hand side of the top fused level (global)
    float* x_top;               // its output x + d (global)
    FusedLv lv[FUSE_MAXLV];
};

// A V-cycle captured from the library's launches and replayed as one HIP
// graph; valid for the hierarchy it was captured from and the key below.
struct VGraph {
    int s = 0, prec = 0;
    const void *z = nullptr, *r64 = nullptr, *q64 = nullptr;
    hipGraphExec_t exec = nullptr;
};

struct MGData {
    int field = 0;              // 0 pressure, 1 velocity component
    int np0 = 0;                // nodes per direction of level 0
    int64_t n0 = 0;             // level-0 DoFs
    double pen = 1.0, wall = -1.0;
    double alpha[3] = {0.0, 0.0, 0.0};
    int degree = 4, lanczos_steps = 15, coarse_cells = 0, max_coarse = 2048;
    double range = 15.0, safety = 1.1;
    std::vector<MGLevel> lv;
    double* ainv[3] = {nullptr, nullptr, nullptr};   // coarse inverses per stage (device, row-major)
    double* z = nullptr;        // FP64 preconditioned residual (pressure: n0; velocity:
                                // every component, velocity layout)
    double* zpart = nullptr;    // partial sums z.r, z.q of the finest smoother step
    double* rpart = nullptr;    // partial sums r.r of the FP64 update
    double* mones = nullptr;    // pressure: M^p 1 (the constant mode of the BF16 cycle)
    double mtot = 0.0;          // 1 . M^p 1
    double* dsum = nullptr;     // partials of the constant-mode sums
    std::vector<void*> allocs;
    std::vector<VGraph> graphs;
    bool no_fuse = false;
    int fuse_from = -1;         // first level of the single-workgroup coarse cycle (-1: none)
    size_t fuse_lds = 0;        // its LDS bytes
};

// Learned / extrapolated initial guesses of the Helmholtz solves in a step.
struct GuessState {
    tbdg_net* net = nullptr;
    // newest pressure increments, inc[0] the newest: inc[0], inc[2], inc[4]
    // of the stage solved last, inc[1], inc[3], inc[5] of the other stage
    // (one step apart)
    static constexpr int kHist = 6;
    double* inc[kHist] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    double beta[kHist] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0}; // stage weights of those solves
    int n = 0;                              // valid increments
    double* cells = nullptr;               // cell statistics [7][Nc] (also the Gram rows)
    double* partial = nullptr;
    double* sc = nullptr;                   // s_inc, s_div
    double* trial = nullptr;               // learned guess (N_p)
    float* feat = nullptr;                  // network input [6][Nc]
    float* y = nullptr;                     // network output [2][Nc]
    bool feat_valid = false;
    double last_r[2] = {0.0, 0.0};          // residual norms of the last learned / fallback guesses
    float* rec = nullptr;                   // recorded samples [cap][12][Nc] (caller's memory)
    int rec_cap = 0, rec_count = 0;
    std::vector<void*> allocs;
};

// Voxel grid of the guess network: nx * ny * nz voxels per sample, B samples.
struct NetGeo {
    int nx, ny, nz, nvox, B;
};

// Slices of the library's static device scratch array (noalloc.hip) that
// stand in for a context's CG and reduction workspaces.
struct NoallocScratch {
    double *cr, *cp, *cq, *cp2;
    double* red_part;
    int red_blocks;
    double* red_out;
    double* red_op;
    int64_t red_op_len;
};

}  // namespace trbdg

struct tbdg_ctx {
    int dim = 0, k = 0, n = 0, np = 0;
    int device = 0;     // HIP device current at create
    // time scheme of tbdg_step (TBDG_SCHEME_*); the single-stage schemes keep
    // their (beta, theta) in stage slot 1
    int scheme = TBDG_SCHEME_TRBDF2;
    double* s_wlag = nullptr;   // BDF2: momentum predictor of the last step (lazy)
    bool wlag_valid = false;
    int64_t Nc = 0, nbu = 0, nbp = 0, Nu = 0, Np = 0, Ns = 0;  // Ns = Nu / dim
    trbdg::Geom geom{};
    trbdg::Tables tab{};
    trbdg::LineGeom lgeom{};
    trbdg::Line1D line_u{}, line_p{};
    double nu = 0, c = 0, dt = 0, gamma = 0, pen_u = 1, pen_p = 1;
    double a31 = 0, a32 = 0, a33 = 0;
    double beta[3] = {0, 0, 0}, theta[3] = {0, 0, 0};
    double sig_u[3] = {0, 0, 0}, sig_p[3] = {0, 0, 0};   // penalties per face direction
    double cr_u = 0, cr_p = 0;   // reference-cell penalties (k+1)^2 pen_u, k^2 pen_p
    int periodic_flags[3] = {1, 1, 1};
    hipStream_t stream = nullptr;
    std::string last_error;
    mutable trbdg::KTimer timer;

    // persistent device workspaces
    double* diag_p[3] = {nullptr, nullptr, nullptr};   // pressure diagonals, stage 1/2
    double* diag_u = nullptr;                           // momentum diagonal (Ns)
    // GMRES
    int gm_m = 0;
    double* V = nullptr;        // (m+1) * Nu basis
    double* gv = nullptr;       // Nu scratch
    double* gz = nullptr;       // Nu scratch
    double* gsc = nullptr;      // inverse norms of the Krylov vectors (gm_m + 1)
    float* mom_blk = nullptr;   // inverse line blocks of the momentum preconditioner (FP32, lazy)
    double* mom_dbox = nullptr; // mapped cells: the box diagonal of those blocks (Ns, lazy)
    double* gm_part = nullptr;  // partials of the fused operator dots
    int64_t gm_part_len = 0;
    // CG
    double* cr = nullptr;
    double* cp = nullptr;
    double* cq = nullptr;
    double* cp2 = nullptr;      // second CG direction buffer (ping-pong)
    // reductions
    double* red_part = nullptr;     // partial sums
    int red_blocks = 0;
    double* red_out = nullptr;      // device scalars
    double* red_op = nullptr;       // per-block partials of operator kernels (one slot per block)
    int64_t red_op_len = 0;
    double* invd_u = nullptr;       // 1 / momentum diagonal (Ns)
    double* invd_p[3] = {nullptr, nullptr, nullptr};
    double* host_out = nullptr;     // pinned host mirror (coherent)
    double* host_dev = nullptr;     // device address of host_out: finishing kernels write
                                    // scalars there directly
    // step scratch
    double* s_w = nullptr;
    double* s_rhs = nullptr;
    double* s_ustar = nullptr;
    double* s_ug = nullptr;
    double* s_u1 = nullptr;
    double* s_pb = nullptr;
    double* s_pg = nullptr;
    double* s_p1 = nullptr;
    double* s_pv = nullptr;     // pressure interpolated to velocity nodes (Ns)
    // Dirichlet data: slot 0 at the stage-1 time t^{n+gamma}, slot 1 at t^{n+1}
    // (the single-stage schemes read slot 1)
    double* bnd_uD[2] = {nullptr, nullptr};
    int64_t bnd_npts = 0;
    int64_t bnd_off[3][2] = {{-1, -1}, {-1, -1}, {-1, -1}};
    int bnd_slot(int s) const { return (s == 2 || scheme != TBDG_SCHEME_TRBDF2) ? 1 : 0; }
    trbdg::Bnd bnd(int s) const {
        trbdg::Bnd b{bnd_uD[bnd_slot(s)], {}};
        for (int a = 0; a < 3; ++a)
            for (int k = 0; k < 2; ++k) b.off[a][k] = bnd_off[a][k];
        return b;
    }
    // fully nonlinear stages: at most nl_max momentum solves per stage, early
    // stop on the relative change nl_tol; solves used by the last step
    int nl_max = 1;
    double nl_tol = 0.0;
    int nl_solves[2] = {0, 0};
    // Q1-mapped cells (mapping 1, 2D): vertices [Nc][4][2] and face-to-cell
    // measure ratios [Nc][4] on the device
    int mapped = 0;
    double* map_vtx = nullptr;
    double* map_gr = nullptr;
    trbdg::MGData* mg = nullptr;    // multigrid hierarchy (built on first use)
    trbdg::MGData* mgu = nullptr;   // velocity-component hierarchy (momentum solves, lazy)
    // copies of it for components 1 and 2, whose V-cycles replay on their own
    // streams beside component 0's (fork and join by events; lazy)
    trbdg::MGData* mgu_side[2] = {nullptr, nullptr};
    hipStream_t side_stream[2] = {nullptr, nullptr};
    hipEvent_t ev_fork = nullptr, ev_join[2] = {nullptr, nullptr};
    bool mg_graphs = true;          // replay the solvers' V-cycles as captured HIP graphs
    int lineprec_stage = 0;         // stage the momentum line blocks were last built for
    bool reuse_lineprec = true;     // later fixed-point solves of a stage keep them
    hipStream_t cap_stream = nullptr;  // private stream the captures are recorded on (lazy)
    tbdg_mg_desc mg_desc{};         // parameters of the last tbdg_mg_setup (zeros: defaults)
    trbdg::GuessState* gs = nullptr;   // initial-guess history and network

    double alpha(int s) const;
    double mcoef(int s) const { return 1.0 / (beta[s] * dt); }
};

namespace trbdg {

// ---- launchers implemented in kernels.hip -------------------------------------
void launch_apply_pressure(const tbdg_ctx* c, double alpha, const double* p, double* y);
void launch_diag_pressure(const tbdg_ctx* c, double alpha, double* d);
// momentum operator / diagonal of stage s (Dirichlet data of that stage)
void launch_apply_momentum(const tbdg_ctx* c, int s, const double* w, const double* u, double* y);
// r = b - V_s(w) u in one pass where the kernel supports it
void launch_residual_momentum(const tbdg_ctx* c, int s, const double* w, const double* u,
                              const double* b, double* r);
// the same with fused GMRES work; returns the grid size (partials per dot)
int launch_apply_momentum_fused(const tbdg_ctx* c, int s, const double* w, const double* u,
                                double* y, const MomFuse& fz);
void launch_diag_momentum(const tbdg_ctx* c, int s, const double* w, double* d);
// the diagonal of the undistorted box's operator (equal to the above on affine meshes)
void launch_diag_momentum_box(const tbdg_ctx* c, int s, const double* w, double* d);
// line-block preconditioner of the momentum operator: inverse blocks of the
// stage operator (w: advector, d: Jacobi diagonal) and z = P^{-1} (scale v)
void launch_mom_lineblk(const tbdg_ctx* c, int st, const double* w, const double* d,
                        float* blk);
void ensure_mom_blk(tbdg_ctx* c);   // allocates c->mom_blk on first use
// builds the line blocks of stage s for advector w (c->diag_u must hold the
// operator's diagonal) and returns the diagonal the blocks were built with,
// which the apply takes: c->diag_u, or on mapped cells the box diagonal
const double* build_mom_lineprec(tbdg_ctx* c, int s, const double* w);
// z = P^{-1} (s v) (s = *scale when given); with accumulate z += P^{-1} (s v)
void launch_mom_lineprec(const tbdg_ctx* c, const float* blk, const double* d, const double* v,
                         const double* scale, double* z, bool accumulate = false);
// sum-factorised Helmholtz right-hand side
void launch_rhs_p_lines(const tbdg_ctx* c, double alpha, double fcoef, const double* u_ss,
                        const double* p_prev, double* rhs);
// line-structured momentum right-hand side (pv: pressure at the velocity nodes)
void launch_rhs_lines(const tbdg_ctx* c, double mcoef, const double* u_prev, const double* u1,
                      const double* w1, double cd1, double ca1, const double* u2, const double* w2,
                      double cd2, double ca2, const double* pv, double* rhs);
// rhs = m M u_prev + sum_pairs [ -cd L0 u_i + ca A0(w_i) u_i ] + Gw p
void launch_rhs_momentum(const tbdg_ctx* c, double mcoef, const double* u_prev,
                         const double* u1, const double* w1, double cd1, double ca1,
                         const double* u2, const double* w2, double cd2, double ca2,
                         const double* p, double* rhs);
// rhs += Dirichlet-data terms of stage s on every boundary face (advector w)
void launch_dirichlet_rhs(const tbdg_ctx* c, int s, const double* w, double* rhs);
void launch_add_grad_p(const tbdg_ctx* c, const double* x, double a, const double* p, double* y);
void launch_rhs_pressure(const tbdg_ctx* c, double alpha, double fcoef, const double* u_ss,
                         const double* p_prev, double* rhs);
void launch_node_coords(const tbdg_ctx* c, int field, double* xyz);

// Start/stop events for one kernel launched with hipExtLaunchKernelGGL when
// the context's timer is on (the runtime timestamps the dispatch itself, so
// the interval is the kernel's execution); null events otherwise.
class TimedLaunch {
  public:
    TimedLaunch(const tbdg_ctx* c, int which, double bytes);
    ~TimedLaunch();
    hipEvent_t start() const { return e1_; }
    hipEvent_t stop() const { return e2_; }
  private:
    const tbdg_ctx* c_;
    int which_;
    hipEvent_t e1_ = nullptr, e2_ = nullptr;
};
void timer_collect(const tbdg_ctx* c);
void timer_release(const tbdg_ctx* c);

// ---- Q1-mapped cells (mapped.hip) ------------------------------------------------
// pressure operator, mode 0 (apply), 3 (fused CG step) or 4 (fused flexible
// CG step) with the arguments of the affine fused kernels; *G_out = blocks
void map_apply_pressure(const tbdg_ctx* c, double alpha, const double* p, double* y, int mode,
                        double* partial, const double* r, const double* invd, double* sc,
                        double* p_out, const double* up, int Gu, int first, int slot,
                        int slot_prev, int* G_out);
void map_diag_pressure(const tbdg_ctx* c, double alpha, double* d);
int map_apply_momentum(const tbdg_ctx* c, int st, const double* w, const double* u, double* y,
                       const MomFuse& fz);
void map_diag_momentum(const tbdg_ctx* c, int st, const double* w, double* d);
void map_rhs_momentum(const tbdg_ctx* c, double mcoef, const double* u_prev, const double* u1,
                      const double* w1, double cd1, double ca1, const double* u2, const double* w2,
                      double cd2, double ca2, const double* p, double* rhs);
void map_dirichlet_rhs(const tbdg_ctx* c, int s, const double* w, double* rhs);
void map_rhs_pressure(const tbdg_ctx* c, double alpha, double fcoef, const double* u_ss,
                      const double* p_prev, double* rhs);
void map_add_grad_p(const tbdg_ctx* c, const double* x, double a, const double* p, double* y);
void map_node_coords(const tbdg_ctx* c, int field, double* xyz);
// host set-up of the mapped geometry (setup.cpp): vertices and measure ratios
void build_mapped_geometry(const tbdg_ctx* c, double amp, std::vector<double>& vtx,
                           std::vector<double>& gr);

// ---- vector kernels implemented in blas.hip -------------------------------------
void vec_axpby(hipStream_t s, int64_t n, double a, const double* x, double b, const double* y, double* out);
void vec_scale_copy(hipStream_t s, int64_t n, double a, const double* x, double* out);
// out[i] = x[i] / d[i % period... ] helpers
void vec_div_diag_u(hipStream_t s, int64_t n, int dim, int64_t nb, const double* x,
                    const double* d, double* out);
void vec_div(hipStream_t s, int64_t n, const double* x, const double* d, double* out);
// device dot products: results written to dev_out[0..k-1]
void dot_many(tbdg_ctx* c, int64_t n, int k, const double* V, int64_t ldv, const double* w,
              double* dev_out);
void dot2(tbdg_ctx* c, int64_t n, const double* a, const double* b, double* dev_out);
// w -= V h (h on device, k vectors)
void vec_sub_combo(hipStream_t s, int64_t n, int k, const double* V, int64_t ldv,
                   const double* h, double* w);
// x += V y (y on device)
void vec_add_combo(hipStream_t s, int64_t n, int k, const double* V, int64_t ldv,
                   const double* y, const double* gsc, double* x);

// ---- CG building blocks (blas.hip) --------------------------------------------
// CG scalars on the device, sc[0] = rz, sc[1] = pAp, sc[2] = rr, sc[3] = rz_new,
// sc[4] = alpha, sc[5] = beta, sc[6] = breakdown flag
void cg_alpha(tbdg_ctx* c, int64_t n, const double* p, const double* q, double* sc);
void cg_update(tbdg_ctx* c, int64_t n, const double* diag, double* x, double* r,
               const double* p, const double* q, double* sc);
void cg_direction(hipStream_t s, int64_t n, const double* diag, const double* r, double* p,
                  const double* sc);
void cg_init(tbdg_ctx* c, int64_t n, const double* diag, const double* r, double* p, double* sc);
void vec_recip(hipStream_t s, int64_t n, const double* d, double* out);
void cg_start(tbdg_ctx* c, int64_t n, const double* invd, const double* r, double* p, double* sc,
              double* up, int Gu);
void cg_dir(tbdg_ctx* c, int64_t n, const double* invd, const double* r, double* p, const double* sc);
void cg_upd(tbdg_ctx* c, int64_t n, const double* invd, double* x, double* r, const double* p,
            const double* q, double* sc, const double* pa, int Ga, int slot, double* up, int Gu);
void cg_alpha_finish(const tbdg_ctx* c, int G, const double* partial, double* sc);
// One fused CG operator step (beta from the update kernel's partials `up`,
// p_new = r invd + beta p_old, q = H p_new, per-block p_new . q partials in
// c->red_op); returns the number of partials.  p_new must not alias p_old.
int launch_cg_apply(const tbdg_ctx* c, double alpha, const double* r, const double* invd,
                    const double* p_old, double* p_new, double* q, double* sc, const double* up,
                    int Gu, int first, int slot, int slot_prev);
// GMRES with unnormalised Krylov vectors V_i and their inverse norms gsc[i]
// kept on the device.  gm_dots: dev_out[i] = gsc_i (V_i . w), i < k, and
// dev_out[k] = w . w; gm_finish_dots: the same from the partials of the fused
// operator kernel.  gm_update_norm: w -= sum_i dev h_i gsc_i V_i, dev_nn =
// |w|^2, gsc_next = 1 / |w| (1 if zero).  gm_norm_inv: dev_nn = |v|^2 and
// inv = 1 / |v|.
// Every finishing step also writes its scalars to host_out (through host_dev)
// at the same offsets as in red_out, so the host only synchronises.
void gm_dots(tbdg_ctx* c, int64_t n, int k, const double* V, int64_t ldv, const double* w,
             const double* gsc, double* dev_out);
void gm_finish_dots(tbdg_ctx* c, int G, int k, const double* part, const double* gsc,
                    double* dev_out);
void gm_update_norm(tbdg_ctx* c, int64_t n, int k, const double* V, int64_t ldv, const double* h,
                    const double* gsc, double* w, double* dev_nn, double* gsc_next);
void gm_norm_inv(tbdg_ctx* c, int64_t n, const double* v, double* dev_nn, double* inv);
// restart without an operator apply (with xcomb: xcomb = sum_{j<k} y_j gsc_j V_j
// instead of the update of x): x += D^{-1} sum_{j<k} y_j gsc_j V_j,
// V_0 = sum_{j<=k} cr_j gsc_j V_j; dev_nn = |V_0|^2, gsc0 = 1 / |V_0|
void gm_restart(tbdg_ctx* c, int64_t n, int k, double* V, int64_t ldv, const double* y,
                const double* cr, const double* gsc, const double* invd, double* x, double* dev_nn,
                double* gsc0, double* xcomb = nullptr);
// x += gz / diag (velocity layout)
void vec_add_div_diag_u(hipStream_t s, int64_t n, int dim, int64_t nb, const double* gz,
                        const double* d, double* x);


// ---- pressure operator on any multigrid level (lines.hip) -------------------------
void launch_pressure_level(hipStream_t s, int dim, int np, const Geom& g, const LineGeom& lg,
                           const Line1D& lt, const Tables& t, double cr, double cm,
                           const double* p, double* y, int64_t Nc);
void launch_diag_pressure_level(hipStream_t s, int dim, int np, const Geom& g, const LineGeom& lg,
                                const Line1D& lt, const Tables& t, double cm, double* d,
                                int64_t Nc);
// One fused flexible-CG operator step: p_new = z + sc[5] p_old, q = H p_new,
// per-block p_new . q partials in c->red_op; returns the number of partials.
int launch_fcg_apply(const tbdg_ctx* c, double alpha, const double* z, const double* p_old,
                     double* p_new, double* q, double* sc);

// ---- multigrid kernels (mg.hip) ---------------------------------------------------
// MG_ZFIN: z, r64, q64 hold zs values per cell (the level's NB consecutive
// ones are used); r64 and q64 may be null (no partial sums), partial too.
template <typename S>
int launch_level_step(hipStream_t st, int dim, const MGLevel& L, int stage, int mode, float c1,
                      float c2, const S* dop, S* x, S* r, const S* b, S* dout, double* z,
                      const double* r64, const double* q64, double* partial, int zs = 0);
int level_blocks(int dim, const MGLevel& L);
template <typename S>
void launch_restrict(hipStream_t st, int dim, const MGLevel& F, const MGLevel& C, int stage,
                     float c2, const S* rf, bool with_d0);
template <typename S>
void launch_prolong(hipStream_t st, int dim, const MGLevel& F, const MGLevel& C, S* xf,
                    const float* dc);
void launch_coarse(hipStream_t st, const double* Ainv, const float* b, float* x, int n);
template <typename S>
int launch_mg_prep(hipStream_t st, int64_t n, int update, const double* pa, int Ga, double* sc,
                   int slot, double* x, double* r, const double* p, const double* q, S* b0, S* d0,
                   const float* invd, float c2, double* partial);
void launch_mg_beta(hipStream_t st, const double* partial, int G, double* sc, int first, int slot,
                    int slot_prev);
// z += gamma 1 with the exact constant mode (see mg.hip), and the z.r, z.q
// partials of flexible CG recomputed into zpart; returns their count
int launch_deflate(hipStream_t st, int64_t n, double alpha, double mtot, const double* m,
                   const double* r, const double* q, double* z, double* sums, double* zpart,
                   int max_blocks);
// x += g 1, r -= g alpha m with g = (1.r) / (alpha 1.m): the residual's
// constant mode solved exactly (start of a BF16 solve)
void launch_deflate_start(hipStream_t st, int64_t n, double alpha, double mtot, const double* m,
                          double* x, double* r, double* sums);
// the coarse end of a V-cycle in one workgroup (levels fc.lv[0..nlev-1])
void launch_fused_cycle(hipStream_t st, int dim, const FusedCycle& fc, size_t lds);
// largest LDS a workgroup may take on the current device (after raising the
// fused kernel's limit to it)
size_t fused_lds_limit(int dim);
// b0 = s v_comp (s = scale, times *sc_dev when given), d0 = c2 D^{-1} b0: the
// level-0 data of one velocity component ([cell][component][node] layout)
void launch_vel_prep(hipStream_t st, int64_t Nc, int nb, int dim, int comp, const double* v,
                     const double* sc_dev, double scale, float* b0, float* d0, const float* invd,
                     float c2);
void vec_mul(hipStream_t st, int64_t n, const double* a, const double* b, double* out);
void vec_unit(hipStream_t st, int64_t n, int64_t j, double* out);
void vec_fill(hipStream_t st, int64_t n, double v, double* out);
void vec_inv_sqrt(hipStream_t st, int64_t n, const double* d, double* out, float* invf);

// ---- set-up helpers (setup.cpp) ---------------------------------------------------
void gauss_legendre(int n, double* x, double* w);
double lagrange_value(const double* z, int n, int j, double x);
void build_line_matrix(int n, const double* W, const double* D, const double* L0, const double* L1,
                       const double* dL0, const double* dL1, double Cr, Line1D& m);
void level_tables(int np, double pen_p, Tables& t, Line1D& line, double& cr);

// ---- guess-network kernels (net.hip) -----------------------------------------------
// mode 1 (last layer) writes nout FP32 outputs per voxel, [b][nout][voxel]
void net_conv(hipStream_t st, const NetGeo& g, int cin, int cout, int mode, const uint16_t* X,
              const uint16_t* Wp, const float* bias, uint16_t* Yb, float* Yf, const uint16_t* mask,
              int nout = 1);
int net_wgrad(hipStream_t st, const NetGeo& g, int cin, int cout, int dys, const uint16_t* X,
              const uint16_t* dY, float* partial, int rows_per_block);
void net_wgrad_reduce(hipStream_t st, const float* partial, int G, int cout, int cin, int cin_real,
                      float* grad, int64_t w_off, int64_t b_off);
void net_pack_fwd(hipStream_t st, const float* theta, int64_t w_off, int cout_real, int cin_real,
                  int cin, int cout, int S, uint16_t* Wp);
void net_pack_bwd(hipStream_t st, const float* theta, int64_t w_off, int cout_real, int cin_real,
                  int cin2, int S, uint16_t* Wt);
void net_copy_bias(hipStream_t st, const float* theta, int64_t b_off, int n, float* b);
void net_to_channel_last(hipStream_t st, const float* x, int B, int C, int nvox, int CP, uint16_t* out);
int net_mse(hipStream_t st, const float* yhat, const float* y, int64_t n, float* dy, double* partial);
int net_quad_loss(hipStream_t st, const float* yhat, const float* gram, int64_t n, int B, float* dy,
                  double* partial);
void net_adam(hipStream_t st, int64_t n, float* theta, const float* g, float* m, float* v, float lr,
              float b1, float b2, float eps, float c1, float c2);

// ---- learned initial guess (guess.hip, guess.cpp, net.cpp) --------------------------
int launch_guess_cells(const tbdg_ctx* c, const double* d1, const double* d2, const double* d0,
                       const double* b, const double* p, double c1, double c0, double cdiv,
                       double alpha, double* cells, double* partial);
void launch_guess_feat(const tbdg_ctx* c, const double* cells, const double* partial, int G,
                       float* feat, double* sc);
void launch_guess_inject(const tbdg_ctx* c, const double* p, const double* d1, const double* d2,
                         const double* d3, const float* y, double* out);
// Gram target [6][Nc] of the blend (rows: 6 Nc doubles of scratch, partial: Nc/256 + 1)
void launch_guess_target(const tbdg_ctx* c, const double* pn, const double* p, const double* d1,
                         const double* d2, const double* d3, double* rows, double* partial,
                         float* out);
void guess_ensure(tbdg_ctx* c);
void guess_free(tbdg_ctx* c);
void guess_reset(tbdg_ctx* c);
// network input [6][Nc] (into the guess state) of the stage-s solve
void guess_features(tbdg_ctx* c, int s, const double* b, const double* p, const double* d0,
                    double beta0, const double* d1, const double* d2);
void guess_inject(tbdg_ctx* c, const double* p, const double* d1, const double* d2, const double* d3,
                  const float* y, double* out);
void guess_target(tbdg_ctx* c, const double* pn, const double* p, const double* d1, const double* d2,
                  const double* d3, float* out);
// writes the initial guess of the stage-s solve to x; returns 0 (previous
// pressure), 1 (rescaled increment) or 2 (learned)
int guess_prepare(tbdg_ctx* c, int s, int mode, const double* b, const double* p_prev, double* x);
void guess_after_solve(tbdg_ctx* c, int s, const double* p_new, const double* p_prev);
// forward pass of the network on one sample of the mesh's cell grid
void net_infer(tbdg_net* net, const float* x, float* y, int nx, int ny, int nz);
hipStream_t net_stream(const tbdg_net* net);

// ---- multigrid host side (mg.cpp) ---------------------------------------------------
// momentum GMRES (solvers.cpp); reuse_prec: a later fixed-point solve of the
// stage whose line blocks were built by the previous one keeps them
tbdg_status solve_momentum(tbdg_ctx* c, int s, const double* w, const double* b, double* x,
                           const tbdg_solver_opts& o, tbdg_solve_info* info, bool reuse_prec = false);
void mg_setup(tbdg_ctx* c, const tbdg_mg_desc* desc);
void mg_free(tbdg_ctx* c);
// z = B r, one V-cycle (precision 1: FP32, 2: BF16 storage on the finest level)
void mg_apply(tbdg_ctx* c, int stage, int precision, const double* r, double* z);
// velocity hierarchy, built on first use with the parameters of the last
// tbdg_mg_setup; z = P^{-1} (s v) with P = theta_s nu H_0 on every component
// (one FP32 V-cycle each), s = *sc_dev when given, else 1
void mgu_ensure(tbdg_ctx* c);
void mgu_free(tbdg_ctx* c);
void mg_apply_velocity(tbdg_ctx* c, int stage, const double* v, const double* sc_dev, double* z,
                       bool accumulate = false);
tbdg_status solve_pressure_mg(tbdg_ctx* c, int s, const double* b, double* x,
                              const tbdg_solver_opts& o, tbdg_solve_info* info);

// ---- static scratch of the allocation-free entry point (noalloc.hip) --------------
// looks up the device address of the scratch array on `device`, which must
// be current; once per device, later calls return at once
void noalloc_init(int device);
NoallocScratch noalloc_scratch(int device);

}  // namespace trbdg
