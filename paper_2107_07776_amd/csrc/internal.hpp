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
};

}  // namespace trbdg

struct tbdg_ctx {
    int dim = 0, k = 0, n = 0, np = 0;
    int64_t Nc = 0, nbu = 0, nbp = 0, Nu = 0, Np = 0, Ns = 0;  // Ns = Nu / dim
    trbdg::Geom geom{};
    trbdg::Tables tab{};
    double nu = 0, c = 0, dt = 0, gamma = 0, pen_u = 1, pen_p = 1;
    double a31 = 0, a32 = 0, a33 = 0;
    double beta[3] = {0, 0, 0}, theta[3] = {0, 0, 0};
    double sig_u[3] = {0, 0, 0}, sig_p[3] = {0, 0, 0};   // penalties per face direction
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
    // CG
    double* cr = nullptr;
    double* cp = nullptr;
    double* cq = nullptr;
    // reductions
    double* red_part = nullptr;     // partial sums
    int red_blocks = 0;
    double* red_out = nullptr;      // device scalars
    double* host_out = nullptr;     // pinned host mirror
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

    double alpha(int s) const;
    double mcoef(int s) const { return 1.0 / (beta[s] * dt); }
};

namespace trbdg {

// ---- launchers implemented in kernels.hip -------------------------------------
void launch_apply_pressure(const tbdg_ctx* c, double alpha, const double* p, double* y);
void launch_diag_pressure(const tbdg_ctx* c, double alpha, double* d);
void launch_apply_momentum(const tbdg_ctx* c, double mcoef, double theta, const double* w,
                           const double* u, double* y);
void launch_diag_momentum(const tbdg_ctx* c, double mcoef, double theta, const double* w,
                          double* d);
// rhs = m M u_prev + sum_pairs [ -cd L0 u_i + ca A0(w_i) u_i ] + Gw p
void launch_rhs_momentum(const tbdg_ctx* c, double mcoef, const double* u_prev,
                         const double* u1, const double* w1, double cd1, double ca1,
                         const double* u2, const double* w2, double cd2, double ca2,
                         const double* p, double* rhs);
void launch_add_grad_p(const tbdg_ctx* c, const double* x, double a, const double* p, double* y);
void launch_rhs_pressure(const tbdg_ctx* c, double alpha, double fcoef, const double* u_ss,
                         const double* p_prev, double* rhs);
void launch_node_coords(const tbdg_ctx* c, int field, double* xyz);

// Brackets one launch with events when the context's timer is on.
class TimedLaunch {
  public:
    TimedLaunch(const tbdg_ctx* c, int which);
    ~TimedLaunch();
  private:
    const tbdg_ctx* c_;
    int which_;
    hipEvent_t e1_ = nullptr;
};
void timer_collect(const tbdg_ctx* c);
void timer_release(const tbdg_ctx* c);

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
                   const double* y, double* x);

// ---- CG building blocks (blas.hip) --------------------------------------------
// CG scalars on the device, sc[0] = rz, sc[1] = pAp, sc[2] = rr, sc[3] = rz_new,
// sc[4] = alpha, sc[5] = beta, sc[6] = breakdown flag
void cg_alpha(tbdg_ctx* c, int64_t n, const double* p, const double* q, double* sc);
void cg_update(tbdg_ctx* c, int64_t n, const double* diag, double* x, double* r,
               const double* p, const double* q, double* sc);
void cg_direction(hipStream_t s, int64_t n, const double* diag, const double* r, double* p,
                  const double* sc);
void cg_init(tbdg_ctx* c, int64_t n, const double* diag, const double* r, double* p, double* sc);
// x += gz / diag (velocity layout)
void vec_add_div_diag_u(hipStream_t s, int64_t n, int dim, int64_t nb, const double* gz,
                        const double* d, double* x);

}  // namespace trbdg
