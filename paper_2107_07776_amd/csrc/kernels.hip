// Matrix-free DG operator kernels for gfx950 (wave64).
//
// Every kernel is cell-centric: a work-group owns CPB whole cells, one thread
// per node of a cell, stages the cell's data in LDS, and evaluates the volume
// terms by one-dimensional contractions (sum factorisation over the tensor
// Gauss nodes) and the face terms of all 2*dim faces of its cells by gathering
// the neighbour's trace from global memory.  Each cell writes only its own
// outputs, so there are no atomics and results are bitwise reproducible.
//
// The forms are those of Sec. 3 of the paper (eq. bilin_diff, eq. trilinear,
// eq. rhs1, the pressure form a_p, F_p and the projection matrix P).  On an
// affine box every cell has the same Jacobian diag(h), so |K| = h_x h_y h_z,
// physical derivatives are reference derivatives / h_a, and a face with normal
// e_a has surface weight (|K| / h_a) * (tangential Gauss weights).
#include "internal.hpp"

namespace trbdg {
namespace {

constexpr int ipow(int b, int e) { return e == 0 ? 1 : b * ipow(b, e - 1); }

template <int DIM, int N>
struct Layout {
    static constexpr int NB = ipow(N, DIM);          // nodes per cell
    static constexpr int NF = ipow(N, DIM - 1);      // nodes per face
    static constexpr int CPB = (256 / NB) > 0 ? (256 / NB) : 1;
    static constexpr int THREADS = CPB * NB;
    // index of the node with coordinate m along direction a and tangential index t
    __device__ static inline int node(int a, int m, int t) {
        if (DIM == 2) return a == 0 ? m + N * t : t + N * m;
        if (a == 0) return m + N * t;
        if (a == 1) return (t % N) + N * m + N * N * (t / N);
        return t + N * N * m;
    }
    __device__ static inline int coord(int nd, int a) {
        return a == 0 ? nd % N : (a == 1 ? (nd / N) % N : nd / (N * N));
    }
    __device__ static inline int tang(int nd, int a) {
        if (DIM == 2) return a == 0 ? nd / N : nd % N;
        if (a == 0) return nd / N;
        if (a == 1) return (nd % N) + N * (nd / (N * N));
        return nd % (N * N);
    }
};

// Neighbour of cell c across face (a, s); -1 on a non-periodic boundary.
template <int DIM>
__device__ inline int64_t neighbor(const Geom& g, const int* per, int64_t c, int a, int s) {
    int64_t ci[3];
    int64_t r = c;
    for (int b = 0; b < DIM; ++b) {
        ci[b] = r % g.nc[b];
        r /= g.nc[b];
    }
    int64_t x = ci[a] + (s ? 1 : -1);
    if (x < 0 || x >= g.nc[a]) {
        if (!per[a]) return -1;
        x = (x + g.nc[a]) % g.nc[a];
    }
    ci[a] = x;
    int64_t out = 0, stride = 1;
    for (int b = 0; b < DIM; ++b) {
        out += ci[b] * stride;
        stride *= g.nc[b];
    }
    return out;
}

template <int DIM, int N>
__device__ inline double node_weight(const double* W, int nd) {
    double w = 1.0;
    for (int a = 0; a < DIM; ++a) w *= W[Layout<DIM, N>::coord(nd, a)];
    return w;
}

template <int DIM, int N>
__device__ inline double tang_weight(const double* W, int t) {
    return DIM == 2 ? W[t] : W[t % N] * W[t / N];
}

struct Periodic {
    int p[3];
};

// ============================================================================
// Pressure interpolated to the velocity nodes (exact: Q_{k-1} is contained in
// the span of the velocity Lagrange basis).  pv: [cell][velocity node].
// ============================================================================
template <int DIM, int N>
__device__ inline double interp_p_at(const Tables& t, const double* pc, int nd) {
    constexpr int NP = N - 1;
    constexpr int NBP = ipow(NP, DIM);
    using Lay = Layout<DIM, N>;
    using LayP = Layout<DIM, NP>;
    double v = 0.0;
    for (int j = 0; j < NBP; ++j) {
        double b = 1.0;
        for (int a = 0; a < DIM; ++a) b *= t.Ip[Lay::coord(nd, a) * NMAX + LayP::coord(j, a)];
        v += b * pc[j];
    }
    return v;
}

// Dirichlet-data terms of the momentum functionals on the boundary faces
// normal to direction a, per component c and face point (eq. rhs1 and its
// stage-2 analogue with the stage's theta and data):
//   -theta nu int u_D,c (n.grad v) + theta nu int 2 C u_D,c v
//   - theta int u_D,c (w.n) v + theta int lambda u_D,c v,
// lambda = max(|w.n|, |(2 u_D - w).n|).  One thread per (boundary cell of
// the face, face point, component) handles both sides of its cell, so two
// threads never add to the same entry; directions are separate launches.
template <int DIM, int N>
__global__ __launch_bounds__(256) void k_dirichlet_rhs(Geom g, Tables t, Bnd bd, int a, double tnu,
                                                        double th, double two_c,
                                                        const double* __restrict__ w,
                                                        double* __restrict__ rhs, int64_t ncells_face) {
    using Lay = Layout<DIM, N>;
    constexpr int NB = Lay::NB, NF = Lay::NF;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= ncells_face * NF * DIM) return;
    const int c = (int)(gid % DIM);
    const int tt = (int)((gid / DIM) % NF);
    const int64_t tc = gid / (DIM * NF);
    // coordinates of the boundary cell: tc enumerates the other directions
    int64_t ci[3] = {0, 0, 0};
    {
        int64_t r = tc;
        for (int b = 0; b < DIM; ++b) {
            if (b == a) continue;
            ci[b] = r % g.nc[b];
            r /= g.nc[b];
        }
    }
    const double inv_h = 1.0 / g.h[a];
    const double wf = g.vol * inv_h * tang_weight<DIM, N>(t.Wu, tt);
    for (int side = 0; side < 2; ++side) {
        ci[a] = side ? g.nc[a] - 1 : 0;
        const int64_t cell = ci[0] + (int64_t)g.nc[0] * (ci[1] + (int64_t)g.nc[1] * ci[2]);
        const double* Ls = side ? t.L1u : t.L0u;
        const double* dLs = side ? t.dL1u : t.dL0u;
        const double sg = side ? 1.0 : -1.0;
        double wa = 0.0;
#pragma unroll
        for (int m = 0; m < N; ++m) wa += Ls[m] * w[(cell * DIM + a) * NB + Lay::node(a, m, tt)];
        const int64_t pt = bd.off[a][side] + tc * NF + tt;
        const double uDa = bd.uD[pt * DIM + a], uDc = bd.uD[pt * DIM + c];
        const double lam = fmax(fabs(wa), fabs(2.0 * uDa - wa));
        const double cv = tnu * two_c - th * sg * wa + th * lam;    // multiplies v on the face
        const double cg = -tnu * sg * inv_h;                        // multiplies l_m' at the face
#pragma unroll
        for (int m = 0; m < N; ++m)
            rhs[(cell * DIM + c) * NB + Lay::node(a, m, tt)] += wf * uDc * (cv * Ls[m] + cg * dLs[m]);
    }
}

template <int DIM, int N>
__global__ __launch_bounds__(256) void k_interp_p(Tables t, const double* __restrict__ p,
                                                   double* __restrict__ pv, int64_t Nc) {
    constexpr int NB = ipow(N, DIM);
    constexpr int NBP = ipow(N - 1, DIM);
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= Nc * NB) return;
    const int64_t cell = gid / NB;
    const int nd = (int)(gid % NB);
    pv[gid] = interp_p_at<DIM, N>(t, p + cell * NBP, nd);
}

// y = x + a * (grad p at velocity nodes)
template <int DIM, int N>
__global__ __launch_bounds__(256) void k_add_grad_p(Geom g, Tables t, const double* x, double a,
                                                     const double* __restrict__ p, double* y,
                                                     int64_t Nc) {
    // y = x + a grad p at the velocity nodes, sum-factorised: each thread
    // takes its node's rows of the 1D pressure basis (values I, derivatives
    // D) once and contracts the cell's pressure direction by direction
    constexpr int NP = N - 1;
    constexpr int NB = ipow(N, DIM);
    constexpr int NBP = ipow(NP, DIM);
    using Lay = Layout<DIM, N>;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= Nc * NB) return;
    const int64_t cell = gid / NB;
    const int nd = (int)(gid % NB);
    const double* pc = p + cell * NBP;
    double I[DIM][NP], D[DIM][NP];
#pragma unroll
    for (int e = 0; e < DIM; ++e) {
        const int ie = Lay::coord(nd, e);
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            I[e][j] = t.Ip[ie * NMAX + j];
            D[e][j] = t.Dpu[ie * NMAX + j];
        }
    }
    double gr[DIM];
    if (DIM == 2) {
        double gx = 0.0, gy = 0.0;
#pragma unroll
        for (int jy = 0; jy < NP; ++jy) {
            double sd = 0.0, si = 0.0;
#pragma unroll
            for (int jx = 0; jx < NP; ++jx) {
                const double pv = pc[jx + NP * jy];
                sd += D[0][jx] * pv;
                si += I[0][jx] * pv;
            }
            gx += I[1][jy] * sd;
            gy += D[1][jy] * si;
        }
        gr[0] = gx;
        gr[1] = gy;
    } else {
        double gx = 0.0, gy = 0.0, gz = 0.0;
#pragma unroll
        for (int jz = 0; jz < NP; ++jz) {
            double tx = 0.0, ty = 0.0, ti = 0.0;
#pragma unroll
            for (int jy = 0; jy < NP; ++jy) {
                double sd = 0.0, si = 0.0;
#pragma unroll
                for (int jx = 0; jx < NP; ++jx) {
                    const double pv = pc[jx + NP * (jy + NP * jz)];
                    sd += D[0][jx] * pv;
                    si += I[0][jx] * pv;
                }
                tx += I[1][jy] * sd;
                ty += D[1][jy] * si;
                ti += I[1][jy] * si;
            }
            gx += I[DIM - 1][jz] * tx;
            gy += I[DIM - 1][jz] * ty;
            gz += D[DIM - 1][jz] * ti;
        }
        gr[0] = gx;
        gr[1] = gy;
        gr[DIM - 1] = gz;
    }
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        const int64_t idx = (cell * DIM + c) * NB + nd;
        const double xv = x ? x[idx] : 0.0;
        y[idx] = xv + a * gr[c] / g.h[c];
    }
}

template <int DIM, int N>
__global__ void k_node_coords(Geom g, Tables t, int field, double* xyz, int64_t Nc) {
    const int n = field == 0 ? N : N - 1;
    int nb = 1;
    for (int a = 0; a < DIM; ++a) nb *= n;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= Nc * nb) return;
    const int64_t cell = gid / nb;
    int nd = (int)(gid % nb);
    int64_t r = cell;
    for (int a = 0; a < DIM; ++a) {
        const int64_t ca = r % g.nc[a];
        r /= g.nc[a];
        const int ia = nd % n;
        nd /= n;
        const double xr = field == 0 ? t.xu[ia] : t.xp[ia];
        xyz[gid * DIM + a] = g.lo[a] + (ca + xr) * g.h[a];
    }
}

inline unsigned nblocks(int64_t work, int per) { return (unsigned)((work + per - 1) / per); }

inline Periodic periodic_of(const tbdg_ctx* c) {
    Periodic p{};
    for (int a = 0; a < 3; ++a) p.p[a] = c->periodic_flags[a];
    return p;
}

}  // namespace

// ---------------------------------------------------------------------------
// dispatch on (dim, n = k + 1)
// ---------------------------------------------------------------------------
#define TBDG_DISPATCH(ctx, FN)                                                            \
    do {                                                                                  \
        const int d_ = (ctx)->dim, n_ = (ctx)->n;                                         \
        if (d_ == 2 && n_ == 3) { FN(2, 3); }                                             \
        else if (d_ == 2 && n_ == 4) { FN(2, 4); }                                        \
        else if (d_ == 2 && n_ == 5) { FN(2, 5); }                                        \
        else if (d_ == 2 && n_ == 6) { FN(2, 6); }                                        \
        else if (d_ == 3 && n_ == 3) { FN(3, 3); }                                        \
        else if (d_ == 3 && n_ == 4) { FN(3, 4); }                                        \
        else throw Error(TBDG_EUNSUPPORTED, "unsupported (dim, degree)");                 \
    } while (0)

void launch_rhs_momentum(const tbdg_ctx* c, double mcoef, const double* u_prev,
                         const double* u1, const double* w1, double cd1, double ca1,
                         const double* u2, const double* w2, double cd2, double ca2,
                         const double* p, double* rhs) {
    if (c->mapped) {
        map_rhs_momentum(c, mcoef, u_prev, u1, w1, cd1, ca1, u2, w2, cd2, ca2, p, rhs);
        return;
    }
    double* pv = c->s_pv;
#define L_(D, N)                                                                          \
    {                                                                                     \
        using Lay = Layout<D, N>;                                                         \
        hipLaunchKernelGGL((k_interp_p<D, N>), dim3(nblocks(c->Ns, 256)), dim3(256), 0,   \
                           c->stream, c->tab, p, pv, c->Nc);                              \
    }
    TBDG_DISPATCH(c, L_);
#undef L_
    TBDG_HIP(hipGetLastError());
    launch_rhs_lines(c, mcoef, u_prev, u1, w1, cd1, ca1, u2, w2, cd2, ca2, pv, rhs);
}

void launch_dirichlet_rhs(const tbdg_ctx* c, int s, const double* w, double* rhs) {
    if (c->mapped) {
        map_dirichlet_rhs(c, s, w, rhs);
        return;
    }
    const Bnd bd = c->bnd(s);
    for (int a = 0; a < c->dim; ++a) {
        if (bd.off[a][0] < 0) continue;
        const int64_t ncf = c->Nc / c->geom.nc[a];
        const double two_c = 2.0 * c->cr_u / c->geom.h[a];
#define L_(D, N)                                                                          \
        {                                                                                 \
            using Lay = Layout<D, N>;                                                     \
            hipLaunchKernelGGL((k_dirichlet_rhs<D, N>), dim3(nblocks(ncf * Lay::NF * D, 256)), \
                               dim3(256), 0, c->stream, c->geom, c->tab, bd, a,           \
                               c->theta[s] * c->nu, c->theta[s], two_c, w, rhs, ncf);     \
        }
        TBDG_DISPATCH(c, L_);
#undef L_
        TBDG_HIP(hipGetLastError());
    }
}

void launch_add_grad_p(const tbdg_ctx* c, const double* x, double a, const double* p, double* y) {
    if (c->mapped) {
        map_add_grad_p(c, x, a, p, y);
        return;
    }
#define L_(D, N)                                                                          \
    hipLaunchKernelGGL((k_add_grad_p<D, N>), dim3(nblocks(c->Ns, 256)), dim3(256), 0,     \
                       c->stream, c->geom, c->tab, x, a, p, y, c->Nc);
    TBDG_DISPATCH(c, L_);
#undef L_
    TBDG_HIP(hipGetLastError());
}

void launch_rhs_pressure(const tbdg_ctx* c, double alpha, double fcoef, const double* u_ss,
                         const double* p_prev, double* rhs) {
    if (c->mapped) {
        map_rhs_pressure(c, alpha, fcoef, u_ss, p_prev, rhs);
        return;
    }
    launch_rhs_p_lines(c, alpha, fcoef, u_ss, p_prev, rhs);
}

void launch_node_coords(const tbdg_ctx* c, int field, double* xyz) {
    if (c->mapped) {
        map_node_coords(c, field, xyz);
        return;
    }
    const int64_t n = field == 0 ? c->Ns : c->Np;
#define L_(D, N)                                                                          \
    hipLaunchKernelGGL((k_node_coords<D, N>), dim3(nblocks(n, 256)), dim3(256), 0,        \
                       c->stream, c->geom, c->tab, field, xyz, c->Nc);
    TBDG_DISPATCH(c, L_);
#undef L_
    TBDG_HIP(hipGetLastError());
}

}  // namespace trbdg
