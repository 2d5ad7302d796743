// Kernels on adaptive 2D quadrilateral meshes with hanging nodes.
//
// Every cell is an axis-aligned rectangle of the size of its level, so the
// pressure SIP form a_p (Sec. 3) splits along grid lines as on the uniform
// box: one work item per (cell, direction, line) applies the 1D stiffness
// and the terms of the line's two end faces.  What changes is the exterior
// trace at a face node of the cell (value and normal derivative):
//   same-level neighbour: its trace along the same line;
//   coarser neighbour (this face is half h of its face): the neighbour's
//     face trace, a polynomial along the face, evaluated at this cell's
//     face nodes (tangential interpolation T_h);
//   two finer neighbours: the face integral is the sum of the two fine faces
//     with their own Gauss points; tested against this cell's tangential
//     basis l_t, the exterior part becomes
//       (1 / W_t) sum_h sum_q (w_q / 2) T_h[q][t] (fine trace at q),
//     while the own-trace parts reduce exactly to the node values (the two
//     half rules integrate the degree 2n-2 products exactly).
// The penalty on a face is the average of the two cells' k^2 / h_a.
// Pressure boundary faces carry no term (homogeneous Neumann).
#include <hip/hip_runtime.h>

#include "amr.hpp"
#include "internal.hpp"
#include "lines.hpp"
#include "reduce.hpp"

namespace trbdg {
namespace amr {
namespace {

template <int NP>
__device__ inline int nd2(int a, int m, int t) {
    return a == 0 ? m + NP * t : t + NP * m;
}

// The sum of part[0..G) in every thread of the block, in the order of
// k_amr_finish2 (so bitwise its result): a kernel that consumes a reduction
// of few partials sums them itself instead of waiting for a one-block
// kernel.  Every thread of the block must call it.
__device__ inline double sum_all(const double* part, int G) {
    __shared__ double s_v;
    double a = 0.0;
    for (int i = threadIdx.x; i < G; i += 256) a += part[i];
    a = red::block_sum(a);
    if (threadIdx.x == 0) s_v = a;
    __syncthreads();
    return s_v;
}

// The operand of the pressure kernel at entry i: p itself, or, for the
// fused CG direction, p_new = z + beta p_old formed on the fly
template <bool DIR>
struct Operand {
    const double* __restrict__ z;
    const double* __restrict__ pold;
    double beta;
    __device__ double operator()(size_t i) const {
        if constexpr (DIR) return z[i] + beta * pold[i];
        return z[i];
    }
};

// value and reference normal derivative of cell's trace at side `side` of
// direction a, on the grid line through tangential node tt
template <int NP, class S>
__device__ inline void trace(const S& p, const Tab1& t, int cell, int a, int side, int tt, double& v,
                             double& d) {
    constexpr int NB = NP * NP;
    v = 0.0;
    d = 0.0;
#pragma unroll
    for (int m = 0; m < NP; ++m) {
        const double pv = p((size_t)cell * NB + nd2<NP>(a, m, tt));
        v += t.L[side][m] * pv;
        d += t.dL[side][m] * pv;
    }
}

// y = (alpha M + K) p, or its diagonal (DIAG)
// MODE 0: y = H p; 1: y = diag(H); 2: y = H_own p, the cell-local part of
// H (the exterior traces set to zero): applied to a field that is one unit
// node per cell it returns one column of every cell's diagonal block;
// 3: the CG direction and its product in one pass: p holds z, the new
// direction z + beta p_old (beta = r.z / rz_old, 0 when rz_old is null;
// r.z the scalar *rz_new or the sum of the partials rz_part, which block 0
// then stores in rz_store) is formed for the cell's own nodes, written to
// dir.pnew, and formed again wherever a neighbour's trace reads it;
// y = H p_new.  MODE 0 and 3 write the per-block partial sums of p . y into
// part when it is not null.
template <int NP, int MODE>
__global__ __launch_bounds__(256) void k_amr_pressure(Geo g, Tab1 t, double alpha,
                                                      const double* __restrict__ p,
                                                      double* __restrict__ y, double* part, CgDir dir) {
    constexpr bool DIAG = MODE == 1;
    constexpr bool EXT = MODE == 0 || MODE == 3;
    double beta = 0.0;
    if (MODE == 3) {
        const double rz = dir.rz_part ? sum_all(dir.rz_part, dir.rz_G) : (dir.rz_old ? *dir.rz_new : 0.0);
        if (dir.rz_old) beta = rz / *dir.rz_old;
        if (dir.rz_store && blockIdx.x == 0 && threadIdx.x == 0) *dir.rz_store = rz;
    }
    const Operand<MODE == 3> src{p, (MODE == 3 && dir.rz_old) ? dir.pold : p, beta};
    constexpr int NB = NP * NP;
    constexpr int CPB = 256 / NB;
    __shared__ double s_p[CPB * NB];
    __shared__ double s_e[CPB * 4 * NP * 2];
    __shared__ double s_y[2][CPB * NB];
    const int tid = threadIdx.x;
    const int lc = tid / NB, nd = tid % NB;
    // consecutive cells (and so the neighbours a block gathers) on one XCD
    const int cell0 = lines::xcd_block(blockIdx.x, gridDim.x) * CPB;
    const int cell = cell0 + lc;
    const bool active = lc < CPB && cell < g.Nc;
    if (lc < CPB) s_p[tid] = (active && !DIAG) ? src((size_t)cell * NB + nd) : 0.0;
    if (MODE == 3 && active) dir.pnew[(size_t)cell * NB + nd] = s_p[tid];
    // exterior traces at every face node of the block's cells
    for (int it = tid; it < CPB * 4 * NP; it += 256) {
        const int c2 = it / (4 * NP), f = (it / NP) % 4, tt = it % NP;
        const int cl = cell0 + c2;
        double ve = 0.0, de = 0.0;
        if (EXT && cl < g.Nc) {
            const int meta = g.meta[cl * 4 + f];
            const int kind = meta & 15, half = meta >> 4;
            const int a = f >> 1, s = f & 1, so = 1 - s;
            const int own = g.level[cl];
            if (kind == FACE_SAME) {
                const int nb = g.nbr[cl * 8 + f * 2];
                trace<NP>(src, t, nb, a, so, tt, ve, de);
                de *= (double)(1 << own) / g.H[a];
            } else if (kind == FACE_COARSER) {
                const int nb = g.nbr[cl * 8 + f * 2];
#pragma unroll
                for (int m = 0; m < NP; ++m) {
                    double v, d;
                    trace<NP>(src, t, nb, a, so, m, v, d);
                    ve += t.T[half][tt * NP + m] * v;
                    de += t.T[half][tt * NP + m] * d;
                }
                de *= (double)(1 << (own - 1)) / g.H[a];
            } else if (kind == FACE_FINER) {
                for (int h = 0; h < 2; ++h) {
                    const int nb = g.nbr[cl * 8 + f * 2 + h];
#pragma unroll
                    for (int q = 0; q < NP; ++q) {
                        double v, d;
                        trace<NP>(src, t, nb, a, so, q, v, d);
                        const double wq = 0.5 * t.W[q] * t.T[h][q * NP + tt];
                        ve += wq * v;
                        de += wq * d;
                    }
                }
                ve /= t.W[tt];
                de *= (double)(1 << (own + 1)) / (g.H[a] * t.W[tt]);
            }
        }
        s_e[it * 2] = ve;
        s_e[it * 2 + 1] = de;
    }
    __syncthreads();
    // one item per (cell, direction, line)
    for (int it = tid; it < CPB * 2 * NP; it += 256) {
        const int c2 = it / (2 * NP), a = (it / NP) % 2, tt = it % NP;
        const int cl = cell0 + c2;
        if (cl >= g.Nc) continue;
        const int own = g.level[cl];
        const double sc = 1.0 / (double)(1 << own);
        const double h = g.H[a] * sc, ht = g.H[1 - a] * sc;
        const double Wt = t.W[tt] * ht;
        double pp[NP];
#pragma unroll
        for (int m = 0; m < NP; ++m) pp[m] = s_p[c2 * NB + nd2<NP>(a, m, tt)];
        double pv[2], pn[2], C[2], ve[2], de[2];
        int kind[2];
        const double sig = g.csig / h;
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const double nu = s ? 1.0 : -1.0;
            pv[s] = 0.0;
            pn[s] = 0.0;
#pragma unroll
            for (int j = 0; j < NP; ++j) {
                pv[s] += t.L[s][j] * pp[j];
                pn[s] += t.dL[s][j] * pp[j];
            }
            pn[s] *= nu / h;
            const int f = 2 * a + s;
            kind[s] = g.meta[cl * 4 + f] & 15;
            C[s] = kind[s] == FACE_SAME ? sig
                 : kind[s] == FACE_COARSER ? 0.5 * (sig + 0.5 * sig)
                 : kind[s] == FACE_FINER ? 0.5 * (sig + 2.0 * sig) : 0.0;
            const int e = ((c2 * 4 + f) * NP + tt) * 2;
            ve[s] = s_e[e];
            de[s] = s_e[e + 1];
        }
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            double r = 0.0;
            if (DIAG) {
                r = t.S[i * NP + i] * Wt / h;
            } else {
#pragma unroll
                for (int j = 0; j < NP; ++j) r += t.S[i * NP + j] * pp[j];
                r *= Wt / h;
            }
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                if (kind[s] == FACE_BOUNDARY) continue;
                const double nu = s ? 1.0 : -1.0;
                const double Li = t.L[s][i], dLi = nu * t.dL[s][i] / h;
                if (DIAG) {
                    r += Wt * (-dLi * Li + C[s] * Li * Li);
                } else {
                    r += Wt * (-0.5 * (pn[s] + nu * de[s]) * Li - 0.5 * dLi * (pv[s] - ve[s])
                               + C[s] * (pv[s] - ve[s]) * Li);
                }
            }
            s_y[a][c2 * NB + nd2<NP>(a, i, tt)] = r;
        }
    }
    __syncthreads();
    double py = 0.0;
    if (active) {
        const double sc = 1.0 / (double)(1 << g.level[cell]);
        const double m = alpha * t.W[nd % NP] * t.W[nd / NP] * g.H[0] * g.H[1] * sc * sc;
        const double own = DIAG ? 1.0 : s_p[tid];
        const double v = m * own + s_y[0][tid] + s_y[1][tid];
        y[(size_t)cell * NB + nd] = v;
        py = own * v;
    }
    // optional per-block partial sum of p . y (the CG step length)
    if (EXT && part) {
        py = red::block_sum(py);
        if (threadIdx.x == 0) part[blockIdx.x] = py;
    }
}

// Momentum operator y_c = mc M u_c + tnu A u_c + th C(w) u_c on both
// velocity components: A the SIP form of eq. bilin_diff (Dirichlet walls:
// -grad u.n v - u n.grad v + 2 C u v), C(w) the Lax-Friedrichs form of
// eq. trilinear.  The face phase forms, at each face node of every cell,
// the exterior SIP traces as in the pressure kernel and the whole
// advective flux seen by the cell's own test functions: at its own nodes
// when the neighbour is as fine or coarser (the coarser traces
// interpolated), and on a face with two finer neighbours at the fine
// faces' Gauss points (own traces interpolated there, lambda from the two
// traces at each point), tested against the cell's tangential basis.
template <int N>
__global__ __launch_bounds__(256) void k_amr_momentum(Geo g, Tab1 t, double mc, double tnu, double th,
                                                      const double* __restrict__ w,
                                                      const double* __restrict__ u,
                                                      const double* __restrict__ uD,
                                                      double* __restrict__ y) {
    constexpr int NB = N * N;
    constexpr int CPB = 256 / NB;
    __shared__ double s_u[2][CPB * NB];
    __shared__ double s_w[2][CPB * NB];
    __shared__ double s_e[CPB * 4 * N * 6];
    __shared__ double s_y[2][2][CPB * NB];
    const int tid = threadIdx.x;
    const int lc = tid / NB, nd = tid % NB;
    // consecutive cells (and so the neighbours a block gathers) on one XCD
    const int cell0 = lines::xcd_block(blockIdx.x, gridDim.x) * CPB;
    const int cell = cell0 + lc;
    const bool active = lc < CPB && cell < g.Nc;
    if (lc < CPB) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            s_u[c][tid] = active ? u[((size_t)cell * 2 + c) * NB + nd] : 0.0;
            s_w[c][tid] = active ? w[((size_t)cell * 2 + c) * NB + nd] : 0.0;
        }
    }
    __syncthreads();
    for (int it = tid; it < CPB * 4 * N; it += 256) {
        const int c2 = it / (4 * N), f = (it / N) % 4, tt = it % N;
        const int cl = cell0 + c2;
        double e[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};   // (ve, de, F) per component
        if (cl < g.Nc) {
            const int meta = g.meta[cl * 4 + f];
            const int kind = meta & 15, half = meta >> 4;
            const int a = f >> 1, s = f & 1, so = 1 - s;
            const double nu = s ? 1.0 : -1.0;
            const int own = g.level[cl];
            const int base = c2 * NB;
            // own face traces at own face node m: u_c and w_a
            auto own_trace = [&](int m, double& u0, double& u1, double& wa) {
                u0 = u1 = wa = 0.0;
#pragma unroll
                for (int j = 0; j < N; ++j) {
                    const int q = base + nd2<N>(a, j, m);
                    u0 += t.L[s][j] * s_u[0][q];
                    u1 += t.L[s][j] * s_u[1][q];
                    wa += t.L[s][j] * s_w[a][q];
                }
            };
            // neighbour's traces on its grid line m at its side so: values
            // and reference derivatives of u_c, value of w_a
            auto nbr_trace = [&](int nb, int m, double* v, double* d, double& wa) {
                v[0] = v[1] = d[0] = d[1] = wa = 0.0;
#pragma unroll
                for (int j = 0; j < N; ++j) {
                    const int q = nd2<N>(a, j, m);
                    const double u0 = u[((size_t)nb * 2 + 0) * NB + q];
                    const double u1 = u[((size_t)nb * 2 + 1) * NB + q];
                    v[0] += t.L[so][j] * u0;
                    v[1] += t.L[so][j] * u1;
                    d[0] += t.dL[so][j] * u0;
                    d[1] += t.dL[so][j] * u1;
                    wa += t.L[so][j] * w[((size_t)nb * 2 + a) * NB + q];
                }
            };
            if (kind == FACE_BOUNDARY) {
                double u0, u1, wa;
                own_trace(tt, u0, u1, wa);
                const double uda = uD[((size_t)g.bface[cl * 4 + f] * N + tt) * 2 + a];
                const double lam = fmax(fabs(wa), fabs(2.0 * uda - wa));
                e[2] = lam * u0;
                e[5] = lam * u1;
            } else if (kind == FACE_SAME || kind == FACE_COARSER) {
                double v[2], d[2], we;
                const int nb = g.nbr[cl * 8 + f * 2];
                if (kind == FACE_SAME) {
                    nbr_trace(nb, tt, v, d, we);
                } else {
                    v[0] = v[1] = d[0] = d[1] = we = 0.0;
#pragma unroll
                    for (int m = 0; m < N; ++m) {
                        double vm[2], dm[2], wm;
                        nbr_trace(nb, m, vm, dm, wm);
                        const double T = t.T[half][tt * N + m];
                        v[0] += T * vm[0];
                        v[1] += T * vm[1];
                        d[0] += T * dm[0];
                        d[1] += T * dm[1];
                        we += T * wm;
                    }
                }
                const double hn = g.H[a] / (double)(1 << (kind == FACE_SAME ? own : own - 1));
                double uo[2], wo;
                own_trace(tt, uo[0], uo[1], wo);
                const double lam = fmax(fabs(wo), fabs(we));
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    e[3 * c] = v[c];
                    e[3 * c + 1] = d[c] / hn;
                    e[3 * c + 2] = 0.5 * nu * (uo[c] * wo + v[c] * we) + 0.5 * lam * (uo[c] - v[c]);
                }
            } else if (kind == FACE_FINER) {
                const double hn = g.H[a] / (double)(1 << (own + 1));
                double tr0[N], tr1[N], trw[N];
#pragma unroll
                for (int m = 0; m < N; ++m) own_trace(m, tr0[m], tr1[m], trw[m]);
                for (int h = 0; h < 2; ++h) {
                    const int nb = g.nbr[cl * 8 + f * 2 + h];
#pragma unroll
                    for (int q = 0; q < N; ++q) {
                        double v[2], d[2], we;
                        nbr_trace(nb, q, v, d, we);
                        double uo0 = 0.0, uo1 = 0.0, wo = 0.0;
#pragma unroll
                        for (int m = 0; m < N; ++m) {
                            const double T = t.T[h][q * N + m];
                            uo0 += T * tr0[m];
                            uo1 += T * tr1[m];
                            wo += T * trw[m];
                        }
                        const double lam = fmax(fabs(wo), fabs(we));
                        const double wq = 0.5 * t.W[q] * t.T[h][q * N + tt];
                        const double F0 = 0.5 * nu * (uo0 * wo + v[0] * we) + 0.5 * lam * (uo0 - v[0]);
                        const double F1 = 0.5 * nu * (uo1 * wo + v[1] * we) + 0.5 * lam * (uo1 - v[1]);
                        e[0] += wq * v[0];
                        e[1] += wq * d[0];
                        e[2] += wq * F0;
                        e[3] += wq * v[1];
                        e[4] += wq * d[1];
                        e[5] += wq * F1;
                    }
                }
                const double iw = 1.0 / t.W[tt];
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    e[3 * c] *= iw;
                    e[3 * c + 1] *= iw / hn;
                    e[3 * c + 2] *= iw;
                }
            }
        }
#pragma unroll
        for (int q = 0; q < 6; ++q) s_e[it * 6 + q] = e[q];
    }
    __syncthreads();
    // one item per (cell, direction, component, line)
    for (int it = tid; it < CPB * 4 * N; it += 256) {
        const int c2 = it / (4 * N), a = (it / (2 * N)) % 2, c = (it / N) % 2, tt = it % N;
        const int cl = cell0 + c2;
        if (cl >= g.Nc) continue;
        const int own = g.level[cl];
        const double sc = 1.0 / (double)(1 << own);
        const double h = g.H[a] * sc, ht = g.H[1 - a] * sc;
        const double Wt = t.W[tt] * ht;
        double pp[N], wa[N];
#pragma unroll
        for (int m = 0; m < N; ++m) {
            const int q = c2 * NB + nd2<N>(a, m, tt);
            pp[m] = s_u[c][q];
            wa[m] = s_w[a][q];
        }
        const double sig = g.csig_u / h;
        double pv[2], pn[2], C[2], ve[2], de[2], F[2];
        int kind[2];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const double nu = s ? 1.0 : -1.0;
            pv[s] = 0.0;
            pn[s] = 0.0;
#pragma unroll
            for (int j = 0; j < N; ++j) {
                pv[s] += t.L[s][j] * pp[j];
                pn[s] += t.dL[s][j] * pp[j];
            }
            pn[s] *= nu / h;
            const int f = 2 * a + s;
            kind[s] = g.meta[cl * 4 + f] & 15;
            C[s] = kind[s] == FACE_SAME ? sig
                 : kind[s] == FACE_COARSER ? 0.5 * (sig + 0.5 * sig)
                 : kind[s] == FACE_FINER ? 0.5 * (sig + 2.0 * sig) : sig;
            const int e = (((c2 * 4 + f) * N + tt) * 6) + 3 * c;
            ve[s] = s_e[e];
            de[s] = s_e[e + 1];
            F[s] = s_e[e + 2];
        }
#pragma unroll
        for (int i = 0; i < N; ++i) {
            double rd = 0.0, ra = 0.0;
#pragma unroll
            for (int j = 0; j < N; ++j) {
                rd += t.S[i * N + j] * pp[j];
                ra -= t.W[j] * t.D[j * N + i] * pp[j] * wa[j];
            }
            rd *= Wt / h;
            ra *= Wt;
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const double nu = s ? 1.0 : -1.0;
                const double Li = t.L[s][i], dLi = nu * t.dL[s][i] / h;
                if (kind[s] == FACE_BOUNDARY)
                    rd += Wt * (-pn[s] * Li - dLi * pv[s] + 2.0 * C[s] * pv[s] * Li);
                else
                    rd += Wt * (-0.5 * (pn[s] + nu * de[s]) * Li - 0.5 * dLi * (pv[s] - ve[s])
                                + C[s] * (pv[s] - ve[s]) * Li);
                ra += Wt * Li * F[s];
            }
            s_y[c][a][c2 * NB + nd2<N>(a, i, tt)] = tnu * rd + th * ra;
        }
    }
    __syncthreads();
    if (active) {
        const double sc = 1.0 / (double)(1 << g.level[cell]);
        const double m = mc * t.W[nd % N] * t.W[nd / N] * g.H[0] * g.H[1] * sc * sc;
#pragma unroll
        for (int c = 0; c < 2; ++c)
            y[((size_t)cell * 2 + c) * NB + nd] = m * s_u[c][tid] + s_y[c][0][tid] + s_y[c][1][tid];
    }
}

// Explicit momentum functional of a stage (eq. rhs1 and its stage-2
// analogue) on both components, see launch_amr_explicit.  The face phase
// forms per face node: the exterior normal derivatives (L0), the whole
// central flux {{u w}}.n seen by the cell's test functions (A0; on coarse
// sides at the fine faces' points), and the own and exterior pressure
// traces at the velocity face points (Gw); on walls the interior traces and
// the wall data.
template <int N>
__global__ __launch_bounds__(256) void k_amr_explicit(Geo g, Tab1 t, MixTab x, ExplicitArgs ea,
                                                      double* __restrict__ y) {
    constexpr int NB = N * N;
    constexpr int NP = N - 1;
    constexpr int NBP = NP * NP;
    constexpr int CPB = 256 / NB;
    __shared__ double s_u[2][CPB * NB];
    __shared__ double s_w[2][CPB * NB];
    __shared__ double s_pu[CPB * NB];     // pressure at the velocity nodes
    __shared__ double s_e[CPB * 4 * N * 6];
    __shared__ double s_y[2][2][CPB * NB];
    const int tid = threadIdx.x;
    const int lc = tid / NB, nd = tid % NB;
    // consecutive cells (and so the neighbours a block gathers) on one XCD
    const int cell0 = lines::xcd_block(blockIdx.x, gridDim.x) * CPB;
    const int cell = cell0 + lc;
    const bool active = lc < CPB && cell < g.Nc;
    if (lc < CPB) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            s_u[c][tid] = active ? ea.ue[((size_t)cell * 2 + c) * NB + nd] : 0.0;
            s_w[c][tid] = active ? ea.we[((size_t)cell * 2 + c) * NB + nd] : 0.0;
        }
        double pu = 0.0;
        if (active && ea.p) {
            const int ix = nd % N, iy = nd / N;
            for (int my = 0; my < NP; ++my) {
                double row = 0.0;
                for (int mx = 0; mx < NP; ++mx) row += x.I[ix * NP + mx] * ea.p[(size_t)cell * NBP + mx + NP * my];
                pu += x.I[iy * NP + my] * row;
            }
        }
        s_pu[tid] = pu;
    }
    __syncthreads();
    for (int it = tid; it < CPB * 4 * N; it += 256) {
        const int c2 = it / (4 * N), f = (it / N) % 4, tt = it % N;
        const int cl = cell0 + c2;
        double e[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        if (cl < g.Nc) {
            const int meta = g.meta[cl * 4 + f];
            const int kind = meta & 15, half = meta >> 4;
            const int a = f >> 1, s = f & 1, so = 1 - s;
            const double nu = s ? 1.0 : -1.0;
            const int own = g.level[cl];
            const int base = c2 * NB;
            auto own_trace = [&](int m, double& u0, double& u1, double& wa) {
                u0 = u1 = wa = 0.0;
#pragma unroll
                for (int j = 0; j < N; ++j) {
                    const int q = base + nd2<N>(a, j, m);
                    u0 += t.L[s][j] * s_u[0][q];
                    u1 += t.L[s][j] * s_u[1][q];
                    wa += t.L[s][j] * s_w[a][q];
                }
            };
            // pressure trace of `pc` at face side `side`, tangential weights tw
            auto p_trace = [&](int pc, int side, const double* tw) {
                double v = 0.0;
                for (int mt = 0; mt < NP; ++mt) {
                    double l = 0.0;
                    for (int ma = 0; ma < NP; ++ma) {
                        const int pn = a == 0 ? ma + NP * mt : mt + NP * ma;
                        l += x.Lp[side][ma] * ea.p[(size_t)pc * NBP + pn];
                    }
                    v += tw[mt] * l;
                }
                return v;
            };
            auto nbr_trace = [&](int nb, int m, double* v, double* d, double& wa) {
                v[0] = v[1] = d[0] = d[1] = wa = 0.0;
#pragma unroll
                for (int j = 0; j < N; ++j) {
                    const int q = nd2<N>(a, j, m);
                    const double u0 = ea.ue[((size_t)nb * 2 + 0) * NB + q];
                    const double u1 = ea.ue[((size_t)nb * 2 + 1) * NB + q];
                    v[0] += t.L[so][j] * u0;
                    v[1] += t.L[so][j] * u1;
                    d[0] += t.dL[so][j] * u0;
                    d[1] += t.dL[so][j] * u1;
                    wa += t.L[so][j] * ea.we[((size_t)nb * 2 + a) * NB + q];
                }
            };
            const double pown = ea.p ? p_trace(cl, s, x.I + tt * NP) : 0.0;
            if (kind == FACE_BOUNDARY) {
                double u0, u1, wa;
                own_trace(tt, u0, u1, wa);
                e[2] = nu * u0 * wa;
                e[3] = nu * u1 * wa;
                e[5] = pown;
                if (ea.uD) {
                    const size_t pt = (size_t)g.bface[cl * 4 + f] * N + tt;
                    const double ud0 = ea.uD[pt * 2], ud1 = ea.uD[pt * 2 + 1];
                    double wd = 0.0;
#pragma unroll
                    for (int j = 0; j < N; ++j)
                        wd += t.L[s][j] * ea.wd[((size_t)cl * 2 + a) * NB + nd2<N>(a, j, tt)];
                    const double uda = a == 0 ? ud0 : ud1;
                    const double lam = fmax(fabs(wd), fabs(2.0 * uda - wd));
                    e[0] = ud0;
                    e[1] = ud1;
                    e[4] = ea.thd * (-nu * wd + lam);
                }
            } else if (kind == FACE_SAME || kind == FACE_COARSER) {
                double v[2], d[2], we;
                double pe = 0.0;
                const int nb = g.nbr[cl * 8 + f * 2];
                if (kind == FACE_SAME) {
                    nbr_trace(nb, tt, v, d, we);
                    if (ea.p) pe = p_trace(nb, so, x.I + tt * NP);
                } else {
                    v[0] = v[1] = d[0] = d[1] = we = 0.0;
#pragma unroll
                    for (int m = 0; m < N; ++m) {
                        double vm[2], dm[2], wm;
                        nbr_trace(nb, m, vm, dm, wm);
                        const double T = t.T[half][tt * N + m];
                        v[0] += T * vm[0];
                        v[1] += T * vm[1];
                        d[0] += T * dm[0];
                        d[1] += T * dm[1];
                        we += T * wm;
                    }
                    if (ea.p) pe = p_trace(nb, so, x.Ih[half] + tt * NP);
                }
                const double hn = g.H[a] / (double)(1 << (kind == FACE_SAME ? own : own - 1));
                double uo[2], wo;
                own_trace(tt, uo[0], uo[1], wo);
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    e[c] = d[c] / hn;
                    e[2 + c] = 0.5 * nu * (uo[c] * wo + v[c] * we);
                }
                e[4] = pe;
                e[5] = pown;
            } else if (kind == FACE_FINER) {
                const double hn = g.H[a] / (double)(1 << (own + 1));
                double tr0[N], tr1[N], trw[N];
#pragma unroll
                for (int m = 0; m < N; ++m) own_trace(m, tr0[m], tr1[m], trw[m]);
                for (int h = 0; h < 2; ++h) {
                    const int nb = g.nbr[cl * 8 + f * 2 + h];
#pragma unroll
                    for (int q = 0; q < N; ++q) {
                        double v[2], d[2], we;
                        nbr_trace(nb, q, v, d, we);
                        double uo0 = 0.0, uo1 = 0.0, wo = 0.0;
#pragma unroll
                        for (int m = 0; m < N; ++m) {
                            const double T = t.T[h][q * N + m];
                            uo0 += T * tr0[m];
                            uo1 += T * tr1[m];
                            wo += T * trw[m];
                        }
                        const double wq = 0.5 * t.W[q] * t.T[h][q * N + tt];
                        e[0] += wq * d[0];
                        e[1] += wq * d[1];
                        e[2] += wq * 0.5 * nu * (uo0 * wo + v[0] * we);
                        e[3] += wq * 0.5 * nu * (uo1 * wo + v[1] * we);
                        if (ea.p) e[4] += wq * p_trace(nb, so, x.I + q * NP);
                    }
                }
                const double iw = 1.0 / t.W[tt];
                e[0] *= iw / hn;
                e[1] *= iw / hn;
                e[2] *= iw;
                e[3] *= iw;
                e[4] *= iw;
                e[5] = pown;
            }
        }
#pragma unroll
        for (int q = 0; q < 6; ++q) s_e[it * 6 + q] = e[q];
    }
    __syncthreads();
    for (int it = tid; it < CPB * 4 * N; it += 256) {
        const int c2 = it / (4 * N), a = (it / (2 * N)) % 2, c = (it / N) % 2, tt = it % N;
        const int cl = cell0 + c2;
        if (cl >= g.Nc) continue;
        const int own = g.level[cl];
        const double sc = 1.0 / (double)(1 << own);
        const double h = g.H[a] * sc, ht = g.H[1 - a] * sc;
        const double Wt = t.W[tt] * ht;
        const bool gw = ea.p && c == a;
        double pp[N], wa[N], pu[N];
#pragma unroll
        for (int m = 0; m < N; ++m) {
            const int q = c2 * NB + nd2<N>(a, m, tt);
            pp[m] = s_u[c][q];
            wa[m] = s_w[a][q];
            pu[m] = s_pu[q];
        }
        const double sig = g.csig_u / h;
        double pn[2];
        int kind[2];
        const double* ee[2];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const double nu = s ? 1.0 : -1.0;
            pn[s] = 0.0;
#pragma unroll
            for (int j = 0; j < N; ++j) pn[s] += t.dL[s][j] * pp[j];
            pn[s] *= nu / h;
            kind[s] = g.meta[cl * 4 + 2 * a + s] & 15;
            ee[s] = s_e + ((c2 * 4 + 2 * a + s) * N + tt) * 6;
        }
#pragma unroll
        for (int i = 0; i < N; ++i) {
            double rl = 0.0, ra = 0.0, rg = 0.0, rd = 0.0;
#pragma unroll
            for (int j = 0; j < N; ++j) {
                rl += t.S[i * N + j] * pp[j];
                ra += t.W[j] * t.D[j * N + i] * pp[j] * wa[j];
                rg += t.W[j] * t.D[j * N + i] * pu[j];
            }
            rl *= Wt / h;
            ra *= Wt;
            rg *= Wt;
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const double nu = s ? 1.0 : -1.0;
                const double Li = t.L[s][i];
                const double* E = ee[s];
                if (kind[s] == FACE_BOUNDARY) {
                    rl += Wt * (-pn[s] * Li);
                    ra -= Wt * Li * E[2 + c];
                    rg -= Wt * nu * E[5] * Li;
                    if (ea.uD) {
                        const double udc = E[c];
                        rd += Wt * (ea.thd * ea.visc * (-udc * nu * t.dL[s][i] / h + 2.0 * sig * udc * Li)
                                    + udc * Li * E[4]);
                    }
                } else {
                    rl += Wt * (-0.5 * (pn[s] + nu * E[c]) * Li);
                    ra -= Wt * Li * E[2 + c];
                    rg -= Wt * 0.5 * nu * (E[5] + E[4]) * Li;
                }
            }
            double r = ea.cl * rl + ea.ca * ra + rd;
            if (gw) r += ea.cg * rg;
            s_y[c][a][c2 * NB + nd2<N>(a, i, tt)] = r;
        }
    }
    __syncthreads();
    if (active) {
        const double sc = 1.0 / (double)(1 << g.level[cell]);
        const double m = ea.mcoef * t.W[nd % N] * t.W[nd / N] * g.H[0] * g.H[1] * sc * sc;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const size_t gi = ((size_t)cell * 2 + c) * NB + nd;
            double v = s_y[c][0][tid] + s_y[c][1][tid];
            if (ea.uprev) v += m * ea.uprev[gi];
            if (ea.acc) v += y[gi];
            y[gi] = v;
        }
    }
}

// b = alpha M^p p + fcoef D u, D u the bracket of F_p:
// sum_K int u.grad q - sum_E int {{u}}.[[q]] (walls: -int (u.n) q), taken at
// the velocity Gauss points; exterior velocity traces per face node as in
// the momentum kernels (projected onto the tangential velocity basis on
// coarse sides, which integrates the pressure test functions exactly).
template <int N>
__global__ __launch_bounds__(256) void k_amr_rhs_p(Geo g, Tab1 t, MixTab x, double alpha,
                                                   const double* __restrict__ p, double fcoef,
                                                   const double* __restrict__ u, double* __restrict__ b) {
    constexpr int NB = N * N;
    constexpr int NP = N - 1;
    constexpr int NBP = NP * NP;
    constexpr int CPB = 256 / NB;
    __shared__ double s_u[2][CPB * NB];
    __shared__ double s_e[CPB * 4 * N * 2];   // own and exterior normal-component traces
    const int tid = threadIdx.x;
    const int lc = tid / NB, nd = tid % NB;
    // consecutive cells (and so the neighbours a block gathers) on one XCD
    const int cell0 = lines::xcd_block(blockIdx.x, gridDim.x) * CPB;
    const int cell = cell0 + lc;
    if (lc < CPB) {
        const bool act = cell < g.Nc;
#pragma unroll
        for (int c = 0; c < 2; ++c) s_u[c][tid] = act ? u[((size_t)cell * 2 + c) * NB + nd] : 0.0;
    }
    __syncthreads();
    for (int it = tid; it < CPB * 4 * N; it += 256) {
        const int c2 = it / (4 * N), f = (it / N) % 4, tt = it % N;
        const int cl = cell0 + c2;
        double uo = 0.0, ue = 0.0;
        if (cl < g.Nc) {
            const int meta = g.meta[cl * 4 + f];
            const int kind = meta & 15, half = meta >> 4;
            const int a = f >> 1, s = f & 1, so = 1 - s;
#pragma unroll
            for (int j = 0; j < N; ++j) uo += t.L[s][j] * s_u[a][c2 * NB + nd2<N>(a, j, tt)];
            auto nbr_trace = [&](int nb, int m) {
                double v = 0.0;
#pragma unroll
                for (int j = 0; j < N; ++j) v += t.L[so][j] * u[((size_t)nb * 2 + a) * NB + nd2<N>(a, j, m)];
                return v;
            };
            if (kind == FACE_SAME) {
                ue = nbr_trace(g.nbr[cl * 8 + f * 2], tt);
            } else if (kind == FACE_COARSER) {
                const int nb = g.nbr[cl * 8 + f * 2];
#pragma unroll
                for (int m = 0; m < N; ++m) ue += t.T[half][tt * N + m] * nbr_trace(nb, m);
            } else if (kind == FACE_FINER) {
                for (int h = 0; h < 2; ++h) {
                    const int nb = g.nbr[cl * 8 + f * 2 + h];
#pragma unroll
                    for (int q = 0; q < N; ++q) ue += 0.5 * t.W[q] * t.T[h][q * N + tt] * nbr_trace(nb, q);
                }
                ue /= t.W[tt];
            }
        }
        s_e[it * 2] = uo;
        s_e[it * 2 + 1] = ue;
    }
    __syncthreads();
    if (tid < CPB * NBP) {
        const int c2 = tid / NBP, pnode = tid % NBP;
        const int cl = cell0 + c2;
        if (cl < g.Nc) {
            const int own = g.level[cl];
            const double sc = 1.0 / (double)(1 << own);
            const int px = pnode % NP, py = pnode / NP;
            double r = 0.0;
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                const int ia = a == 0 ? px : py, itp = a == 0 ? py : px;
                const double ht = g.H[1 - a] * sc;
                for (int tt = 0; tt < N; ++tt) {
                    const double wt = t.W[tt] * ht * x.I[tt * NP + itp];
                    double v = 0.0;
#pragma unroll
                    for (int m = 0; m < N; ++m)
                        v += t.W[m] * x.DI[m * NP + ia] * s_u[a][c2 * NB + nd2<N>(a, m, tt)];
                    double fsum = 0.0;
#pragma unroll
                    for (int s = 0; s < 2; ++s) {
                        const int f = 2 * a + s;
                        const double nu = s ? 1.0 : -1.0;
                        const int kind = g.meta[cl * 4 + f] & 15;
                        const double* E = s_e + ((c2 * 4 + f) * N + tt) * 2;
                        const double tr = kind == FACE_BOUNDARY ? E[0] : 0.5 * (E[0] + E[1]);
                        fsum -= nu * tr * x.Lp[s][ia];
                    }
                    r += wt * (v + fsum);
                }
            }
            const double hx = g.H[0] * sc, hy = g.H[1] * sc;
            // the pressure Gauss weights are those of the np-point rule: rebuild
            // them from the interpolation identity sum_q W_q l^p_m(z_q) = w^p_m
            double wpx = 0.0, wpy = 0.0;
            for (int q = 0; q < N; ++q) {
                wpx += t.W[q] * x.I[q * NP + px];
                wpy += t.W[q] * x.I[q * NP + py];
            }
            const size_t gi = (size_t)cl * NBP + pnode;
            b[gi] = alpha * wpx * wpy * hx * hy * p[gi] + fcoef * r;
        }
    }
}

// y = x + a grad p at the velocity nodes (M^{-1} P p with the collocated
// velocity mass)
template <int N>
__global__ __launch_bounds__(256) void k_amr_grad(Geo g, MixTab x, const double* __restrict__ xin,
                                                  double a, const double* __restrict__ p,
                                                  double* __restrict__ y) {
    constexpr int NB = N * N;
    constexpr int NP = N - 1;
    constexpr int NBP = NP * NP;
    const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (gid >= (int64_t)g.Nc * NB) return;
    const int cell = (int)(gid / NB), nd = (int)(gid % NB);
    const int ix = nd % N, iy = nd / N;
    const double sc = 1.0 / (double)(1 << g.level[cell]);
    double gx = 0.0, gy = 0.0;
    for (int my = 0; my < NP; ++my) {
        double rx = 0.0, ry = 0.0;
        for (int mx = 0; mx < NP; ++mx) {
            const double pv = p[(size_t)cell * NBP + mx + NP * my];
            rx += x.DI[ix * NP + mx] * pv;
            ry += x.I[ix * NP + mx] * pv;
        }
        gx += x.I[iy * NP + my] * rx;
        gy += x.DI[iy * NP + my] * ry;
    }
    gx /= g.H[0] * sc;
    gy /= g.H[1] * sc;
    const size_t b0 = ((size_t)cell * 2) * NB + nd, b1 = b0 + NB;
    y[b0] = xin[b0] + a * gx;
    y[b1] = xin[b1] + a * gy;
}

// Diagonal of mc M + tnu A (the momentum operator without its advection),
// in the velocity layout [cell][component][node]: the Jacobi scaling of the
// momentum GMRES on adapted meshes.
template <int N>
__global__ __launch_bounds__(256) void k_amr_momentum_diag(Geo g, Tab1 t, double mc, double tnu,
                                                           double* __restrict__ d) {
    constexpr int NB = N * N;
    const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (gid >= (int64_t)g.Nc * NB) return;
    const int cell = (int)(gid / NB), nd = (int)(gid % NB);
    const int own = g.level[cell];
    const double sc = 1.0 / (double)(1 << own);
    double r = mc * t.W[nd % N] * t.W[nd / N] * g.H[0] * g.H[1] * sc * sc;
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const int i = a == 0 ? nd % N : nd / N, tt = a == 0 ? nd / N : nd % N;
        const double h = g.H[a] * sc, ht = g.H[1 - a] * sc;
        const double Wt = t.W[tt] * ht;
        const double sig = g.csig_u / h;
        double ra = t.S[i * N + i] * Wt / h;
        for (int s = 0; s < 2; ++s) {
            const int kind = g.meta[cell * 4 + 2 * a + s] & 15;
            const double nu = s ? 1.0 : -1.0;
            const double Li = t.L[s][i], dLi = nu * t.dL[s][i] / h;
            if (kind == FACE_BOUNDARY) {
                ra += Wt * (-2.0 * dLi * Li + 2.0 * sig * Li * Li);
            } else {
                const double C = kind == FACE_SAME ? sig : kind == FACE_COARSER ? 0.75 * sig : 1.5 * sig;
                ra += Wt * (-dLi * Li + C * Li * Li);
            }
        }
        r += tnu * ra;
    }
    d[((size_t)cell * 2 + 0) * NB + nd] = r;
    d[((size_t)cell * 2 + 1) * NB + nd] = r;
}

// eta_K = (h_x^2 + h_y^2) sum_nodes W |K| omega^2, omega = d_x u_y - d_y u_x
template <int N>
__global__ __launch_bounds__(256) void k_amr_indicator(Geo g, Tab1 t, const double* __restrict__ u,
                                                       double* __restrict__ eta) {
    constexpr int NB = N * N;
    constexpr int CPB = 256 / NB;
    __shared__ double s_u[2][CPB * NB];
    __shared__ double s_w[CPB * NB];
    const int tid = threadIdx.x;
    const int lc = tid / NB, nd = tid % NB;
    const int cell = blockIdx.x * CPB + lc;
    const bool active = lc < CPB && cell < g.Nc;
    if (lc < CPB) {
#pragma unroll
        for (int c = 0; c < 2; ++c) s_u[c][tid] = active ? u[((size_t)cell * 2 + c) * NB + nd] : 0.0;
    }
    __syncthreads();
    if (lc < CPB) {
        double om2 = 0.0;
        if (active) {
            const double sc = 1.0 / (double)(1 << g.level[cell]);
            const double hx = g.H[0] * sc, hy = g.H[1] * sc;
            const int ix = nd % N, iy = nd / N;
            double dxuy = 0.0, dyux = 0.0;
#pragma unroll
            for (int j = 0; j < N; ++j) {
                dxuy += t.D[ix * N + j] * s_u[1][lc * NB + j + N * iy];
                dyux += t.D[iy * N + j] * s_u[0][lc * NB + ix + N * j];
            }
            const double om = dxuy / hx - dyux / hy;
            om2 = t.W[ix] * t.W[iy] * hx * hy * om * om;
        }
        s_w[tid] = om2;
    }
    __syncthreads();
    if (lc < CPB && nd == 0 && active) {
        double sum = 0.0;
        for (int q = 0; q < NB; ++q) sum += s_w[lc * NB + q];
        const double sc = 1.0 / (double)(1 << g.level[cell]);
        const double hx = g.H[0] * sc, hy = g.H[1] * sc;
        eta[cell] = (hx * hx + hy * hy) * sum;
    }
}

// one thread per (new cell, component, node)
template <int N>
__global__ __launch_bounds__(256) void k_amr_transfer(XferMap mp, Tab1 t, int ncomp,
                                                      const double* __restrict__ src,
                                                      double* __restrict__ dst) {
    constexpr int NB = N * N;
    const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t total = (int64_t)mp.Nnew * ncomp * NB;
    if (gid >= total) return;
    const int cell = (int)(gid / (ncomp * NB));
    const int rem = (int)(gid % (ncomp * NB));
    const int comp = rem / NB, nd = rem % NB;
    const int ix = nd % N, iy = nd / N;
    const int kd = mp.kind[cell];
    const int kind = kd & 15, pos = kd >> 4;
    const int* s4 = mp.src + (size_t)cell * 4;
    double v = 0.0;
    if (kind == 0) {
        v = src[((size_t)s4[0] * ncomp + comp) * NB + nd];
    } else if (kind == 1) {
        // the parent's polynomial at this child's node
        const int bx = pos & 1, by = pos >> 1;
        const double* ps = src + ((size_t)s4[0] * ncomp + comp) * NB;
#pragma unroll
        for (int my = 0; my < N; ++my) {
            double row = 0.0;
#pragma unroll
            for (int mx = 0; mx < N; ++mx) row += t.T[bx][ix * N + mx] * ps[mx + N * my];
            v += t.T[by][iy * N + my] * row;
        }
    } else {
        // L2 projection of the four children onto the parent node (ix, iy)
        for (int ch = 0; ch < 4; ++ch) {
            const int dx = ch & 1, dy = ch >> 1;
            const double* cs = src + ((size_t)s4[ch] * ncomp + comp) * NB;
            double acc = 0.0;
#pragma unroll
            for (int qy = 0; qy < N; ++qy) {
                double row = 0.0;
#pragma unroll
                for (int qx = 0; qx < N; ++qx) row += t.W[qx] * t.T[dx][qx * N + ix] * cs[qx + N * qy];
                acc += t.W[qy] * t.T[dy][qy * N + iy] * row;
            }
            v += 0.25 * acc;
        }
        v /= t.W[ix] * t.W[iy];
    }
    dst[((size_t)cell * ncomp + comp) * NB + nd] = v;
}

__global__ __launch_bounds__(256) void k_amr_dot(int64_t n, const double* __restrict__ a,
                                                 const double* __restrict__ b, double* part) {
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        s += a[i] * b[i];
    s = red::block_sum(s);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_amr_dot_finish(const double* part, int G, double* out) {
    double s = 0.0;
    for (int i = threadIdx.x; i < G; i += 256) s += part[i];
    s = red::block_sum(s);
    if (threadIdx.x == 0) *out = s;
}

// one unit node per cell: u[c NB + j] = (j == i)
__global__ __launch_bounds__(256) void k_amr_unit(int64_t nc, int nb, int i, double* u) {
    const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (gid < nc * nb) u[gid] = (int)(gid % nb) == i ? 1.0 : 0.0;
}

// column i of every cell's block: B[c][row][i] = y[c NB + row] (FP64 scratch)
__global__ __launch_bounds__(256) void k_amr_block_col(int64_t nc, int nb, int i, const double* y,
                                                       double* B) {
    const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (gid >= nc * nb) return;
    const int64_t c = gid / nb;
    const int row = (int)(gid % nb);
    B[(c * nb + row) * nb + i] = y[gid];
}

// in-place inverse of every cell's SPD block by Gauss-Jordan elimination
// without pivoting (the diagonal block of an SPD matrix is SPD), stored FP32
template <int NBK>
__global__ __launch_bounds__(64) void k_amr_block_inv(int64_t nc, const double* __restrict__ B,
                                                      float* __restrict__ Binv) {
    const int64_t c = (int64_t)blockIdx.x * 64 + threadIdx.x;
    if (c >= nc) return;
    double a[NBK * NBK], v[NBK * NBK];
    for (int q = 0; q < NBK * NBK; ++q) {
        a[q] = B[c * NBK * NBK + q];
        v[q] = (q / NBK == q % NBK) ? 1.0 : 0.0;
    }
    for (int k = 0; k < NBK; ++k) {
        const double ip = 1.0 / a[k * NBK + k];
        for (int j = 0; j < NBK; ++j) {
            a[k * NBK + j] *= ip;
            v[k * NBK + j] *= ip;
        }
        for (int r = 0; r < NBK; ++r) {
            if (r == k) continue;
            const double fct = a[r * NBK + k];
            for (int j = 0; j < NBK; ++j) {
                a[r * NBK + j] -= fct * a[k * NBK + j];
                v[r * NBK + j] -= fct * v[k * NBK + j];
            }
        }
    }
    for (int q = 0; q < NBK * NBK; ++q) Binv[c * NBK * NBK + q] = (float)v[q];
}

// z = B^{-1} r per cell (FP32 blocks, FP64 vectors and sums); block partial
// sums of r.z and r.r in part[b], part[G + b].  XR: the CG update comes
// first, x += al p and r -= al q with al = *xr.rz / p.q (the scalar *xr.pq
// or the sum of the partials xr.pq_part), and z is formed from the updated r
template <int NBK, bool XR>
__global__ __launch_bounds__(256) void k_amr_block_apply(int64_t nc, const float* __restrict__ Binv,
                                                         double* __restrict__ r,
                                                         double* __restrict__ z, double* part,
                                                         CgUpdate xr) {
    constexpr int CPB = 256 / NBK;
    __shared__ double s_r[CPB * NBK];
    const int tid = threadIdx.x;
    const int lc = tid / NBK, i = tid % NBK;
    const int64_t c = (int64_t)blockIdx.x * CPB + lc;
    const bool act = lc < CPB && c < nc;
    double al = 0.0;
    if (XR) al = *xr.rz / (xr.pq_part ? sum_all(xr.pq_part, xr.pq_G) : *xr.pq);
    double rv = 0.0;
    if (act) {
        const int64_t k = c * NBK + i;
        rv = r[k];
        if (XR) {
            xr.x[k] += al * xr.p[k];
            rv -= al * xr.q[k];
            r[k] = rv;
        }
    }
    if (lc < CPB) s_r[tid] = rv;
    __syncthreads();
    double rz = 0.0, rr = 0.0;
    if (act) {
        double zi = 0.0;
        const float* row = Binv + (c * NBK + i) * NBK;
#pragma unroll
        for (int j = 0; j < NBK; ++j) zi += (double)row[j] * s_r[lc * NBK + j];
        z[c * NBK + i] = zi;
        rz = s_r[tid] * zi;
        rr = s_r[tid] * s_r[tid];
    }
    rz = red::block_sum(rz);
    rr = red::block_sum(rr);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = rz;
        part[gridDim.x + blockIdx.x] = rr;
    }
}

// x += al p, r -= al q, z = r / d, al = *u.rz / p.q (the scalar *u.pq or
// the sum of the partials u.pq_part); per-block partial sums of r.z and r.r
// (grid-stride over a fixed grid)
__global__ __launch_bounds__(256) void k_amr_cg_step(int64_t n, CgUpdate u,
                                                     const double* __restrict__ d,
                                                     double* __restrict__ r,
                                                     double* __restrict__ z, double* part) {
    const double al = *u.rz / (u.pq_part ? sum_all(u.pq_part, u.pq_G) : *u.pq);
    double a = 0.0, b = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        u.x[i] += al * u.p[i];
        const double ri = r[i] - al * u.q[i];
        const double zi = ri / d[i];
        r[i] = ri;
        z[i] = zi;
        a += ri * zi;
        b += ri * ri;
    }
    a = red::block_sum(a);
    b = red::block_sum(b);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = a;
        part[gridDim.x + blockIdx.x] = b;
    }
}

// sums of two rows of G partials into out[0], out[1] (second row optional)
__global__ __launch_bounds__(256) void k_amr_finish2(const double* part, int G, int rows, double* out0,
                                                     double* out1) {
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < G; i += 256) {
        a += part[i];
        if (rows > 1) b += part[G + i];
    }
    a = red::block_sum(a);
    b = red::block_sum(b);
    if (threadIdx.x == 0) {
        *out0 = a;
        if (rows > 1) *out1 = b;
    }
}

// z = r / d elementwise; z may alias r
__global__ __launch_bounds__(256) void k_amr_div(int64_t n, const double* r, const double* d,
                                                 double* z) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    z[i] = r[i] / d[i];
}

__global__ __launch_bounds__(256) void k_amr_maxdiff(int64_t n, const double* __restrict__ a,
                                                     const double* __restrict__ b, double* part) {
    double m = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        m = fmax(m, fabs(a[i] - b[i]));
    __shared__ double s_m[256];
    s_m[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s_m[threadIdx.x] = fmax(s_m[threadIdx.x], s_m[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s_m[0];
}

__global__ __launch_bounds__(256) void k_amr_max_finish(const double* part, int G, double* out) {
    __shared__ double s_m[256];
    double m = 0.0;
    for (int i = threadIdx.x; i < G; i += 256) m = fmax(m, part[i]);
    s_m[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s_m[threadIdx.x] = fmax(s_m[threadIdx.x], s_m[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = s_m[0];
}

inline int blocks(int64_t n) { return (int)((n + 255) / 256); }

}  // namespace

int amr_pressure_blocks(const Geo& g, const Tab1& t) {
    const int cpb = 256 / (t.n * t.n);
    return (g.Nc + cpb - 1) / cpb;
}

void launch_amr_pressure(hipStream_t st, const Geo& g, const Tab1& t, double alpha, const double* p,
                         double* y, bool diag, double* part) {
    launch_amr_pressure_mode(st, g, t, alpha, p, y, diag ? 1 : 0, part);
}

void launch_amr_pressure_mode(hipStream_t st, const Geo& g, const Tab1& t, double alpha,
                              const double* p, double* y, int mode, double* part) {
    launch_amr_pressure_any(st, g, t, alpha, p, y, mode, part, CgDir{});
}

void launch_amr_pressure_dir(hipStream_t st, const Geo& g, const Tab1& t, double alpha, const double* z,
                             const CgDir& dir, double* q, double* part) {
    launch_amr_pressure_any(st, g, t, alpha, z, q, 3, part, dir);
}

void launch_amr_pressure_any(hipStream_t st, const Geo& g, const Tab1& t, double alpha, const double* p,
                             double* y, int mode, double* part, const CgDir& dir) {
    if (g.Nc == 0) return;
#define TBDG_AMR_P(NPV)                                                                       \
    case NPV: {                                                                               \
        constexpr int CPB = 256 / (NPV * NPV);                                                \
        const int G = (g.Nc + CPB - 1) / CPB;                                                 \
        if (mode == 1) hipLaunchKernelGGL((k_amr_pressure<NPV, 1>), dim3(G), dim3(256), 0, st, g, \
                                          t, alpha, p, y, nullptr, dir);                     \
        else if (mode == 2) hipLaunchKernelGGL((k_amr_pressure<NPV, 2>), dim3(G), dim3(256), 0, st, \
                                               g, t, alpha, p, y, nullptr, dir);             \
        else if (mode == 3) hipLaunchKernelGGL((k_amr_pressure<NPV, 3>), dim3(G), dim3(256), 0, st, \
                                               g, t, alpha, p, y, part, dir);                \
        else hipLaunchKernelGGL((k_amr_pressure<NPV, 0>), dim3(G), dim3(256), 0, st, g, t, alpha, \
                                p, y, part, dir);                                            \
        break;                                                                                \
    }
    switch (t.n) {
        TBDG_AMR_P(1)
        TBDG_AMR_P(2)
        TBDG_AMR_P(3)
        TBDG_AMR_P(4)
        TBDG_AMR_P(5)
        TBDG_AMR_P(6)
        TBDG_AMR_P(7)
        default: throw Error(TBDG_EUNSUPPORTED, "pressure nodes per direction must be 1..7");
    }
#undef TBDG_AMR_P
    TBDG_HIP(hipGetLastError());
}

void launch_amr_momentum(hipStream_t st, const Geo& g, const Tab1& t, double mc, double tnu, double th,
                         const double* w, const double* u, const double* uD, double* y) {
    if (g.Nc == 0) return;
#define TBDG_AMR_M(NV)                                                                        \
    case NV: {                                                                                \
        constexpr int CPB = 256 / (NV * NV);                                                  \
        hipLaunchKernelGGL((k_amr_momentum<NV>), dim3((g.Nc + CPB - 1) / CPB), dim3(256), 0, st, \
                           g, t, mc, tnu, th, w, u, uD, y);                                   \
        break;                                                                                \
    }
    switch (t.n) {
        TBDG_AMR_M(2)
        TBDG_AMR_M(3)
        TBDG_AMR_M(4)
        TBDG_AMR_M(5)
        TBDG_AMR_M(6)
        TBDG_AMR_M(7)
        TBDG_AMR_M(8)
        default: throw Error(TBDG_EUNSUPPORTED, "velocity nodes per direction must be 2..8");
    }
#undef TBDG_AMR_M
    TBDG_HIP(hipGetLastError());
}

void launch_amr_explicit(hipStream_t st, const Geo& g, const Tab1& t, const MixTab& x,
                         const ExplicitArgs& e, double* y) {
    if (g.Nc == 0) return;
#define TBDG_AMR_E(NV)                                                                        \
    case NV: {                                                                                \
        constexpr int CPB = 256 / (NV * NV);                                                  \
        hipLaunchKernelGGL((k_amr_explicit<NV>), dim3((g.Nc + CPB - 1) / CPB), dim3(256), 0, st, \
                           g, t, x, e, y);                                                    \
        break;                                                                                \
    }
    switch (t.n) {
        TBDG_AMR_E(2)
        TBDG_AMR_E(3)
        TBDG_AMR_E(4)
        TBDG_AMR_E(5)
        TBDG_AMR_E(6)
        TBDG_AMR_E(7)
        TBDG_AMR_E(8)
        default: throw Error(TBDG_EUNSUPPORTED, "velocity nodes per direction must be 2..8");
    }
#undef TBDG_AMR_E
    TBDG_HIP(hipGetLastError());
}

void launch_amr_rhs_p(hipStream_t st, const Geo& g, const Tab1& t, const MixTab& x, double alpha,
                      const double* p, double fcoef, const double* u, double* b) {
    if (g.Nc == 0) return;
#define TBDG_AMR_R(NV)                                                                        \
    case NV: {                                                                                \
        constexpr int CPB = 256 / (NV * NV);                                                  \
        hipLaunchKernelGGL((k_amr_rhs_p<NV>), dim3((g.Nc + CPB - 1) / CPB), dim3(256), 0, st, g, \
                           t, x, alpha, p, fcoef, u, b);                                      \
        break;                                                                                \
    }
    switch (t.n) {
        TBDG_AMR_R(2)
        TBDG_AMR_R(3)
        TBDG_AMR_R(4)
        TBDG_AMR_R(5)
        TBDG_AMR_R(6)
        TBDG_AMR_R(7)
        TBDG_AMR_R(8)
        default: throw Error(TBDG_EUNSUPPORTED, "velocity nodes per direction must be 2..8");
    }
#undef TBDG_AMR_R
    TBDG_HIP(hipGetLastError());
}

void launch_amr_grad(hipStream_t st, const Geo& g, const Tab1& t, const MixTab& x, const double* xin,
                     double a, const double* p, double* y) {
    const int64_t total = (int64_t)g.Nc * t.n * t.n;
    if (total == 0) return;
#define TBDG_AMR_G(NV)                                                                        \
    case NV:                                                                                  \
        hipLaunchKernelGGL((k_amr_grad<NV>), dim3(blocks(total)), dim3(256), 0, st, g, x, xin, a, \
                           p, y);                                                             \
        break;
    switch (t.n) {
        TBDG_AMR_G(2)
        TBDG_AMR_G(3)
        TBDG_AMR_G(4)
        TBDG_AMR_G(5)
        TBDG_AMR_G(6)
        TBDG_AMR_G(7)
        TBDG_AMR_G(8)
        default: throw Error(TBDG_EUNSUPPORTED, "velocity nodes per direction must be 2..8");
    }
#undef TBDG_AMR_G
    TBDG_HIP(hipGetLastError());
}

void launch_amr_momentum_diag(hipStream_t st, const Geo& g, const Tab1& t, double mc, double tnu,
                              double* d) {
    const int64_t total = (int64_t)g.Nc * t.n * t.n;
    if (total == 0) return;
#define TBDG_AMR_MD(NV)                                                                       \
    case NV:                                                                                  \
        hipLaunchKernelGGL((k_amr_momentum_diag<NV>), dim3(blocks(total)), dim3(256), 0, st, g, t, \
                           mc, tnu, d);                                                       \
        break;
    switch (t.n) {
        TBDG_AMR_MD(2)
        TBDG_AMR_MD(3)
        TBDG_AMR_MD(4)
        TBDG_AMR_MD(5)
        TBDG_AMR_MD(6)
        TBDG_AMR_MD(7)
        TBDG_AMR_MD(8)
        default: throw Error(TBDG_EUNSUPPORTED, "velocity nodes per direction must be 2..8");
    }
#undef TBDG_AMR_MD
    TBDG_HIP(hipGetLastError());
}

void launch_amr_indicator(hipStream_t st, const Geo& g, const Tab1& t, const double* u, double* eta) {
    if (g.Nc == 0) return;
#define TBDG_AMR_I(NV)                                                                        \
    case NV: {                                                                                \
        constexpr int CPB = 256 / (NV * NV);                                                  \
        hipLaunchKernelGGL((k_amr_indicator<NV>), dim3((g.Nc + CPB - 1) / CPB), dim3(256), 0, st, \
                           g, t, u, eta);                                                     \
        break;                                                                                \
    }
    switch (t.n) {
        TBDG_AMR_I(2)
        TBDG_AMR_I(3)
        TBDG_AMR_I(4)
        TBDG_AMR_I(5)
        TBDG_AMR_I(6)
        TBDG_AMR_I(7)
        TBDG_AMR_I(8)
        default: throw Error(TBDG_EUNSUPPORTED, "velocity nodes per direction must be 2..8");
    }
#undef TBDG_AMR_I
    TBDG_HIP(hipGetLastError());
}

void launch_amr_transfer(hipStream_t st, const XferMap& m, const Tab1& t, int ncomp, const double* src,
                         double* dst) {
    const int64_t total = (int64_t)m.Nnew * ncomp * t.n * t.n;
    if (total == 0) return;
#define TBDG_AMR_T(NV)                                                                        \
    case NV:                                                                                  \
        hipLaunchKernelGGL((k_amr_transfer<NV>), dim3(blocks(total)), dim3(256), 0, st, m, t,    \
                           ncomp, src, dst);                                                  \
        break;
    switch (t.n) {
        TBDG_AMR_T(1)
        TBDG_AMR_T(2)
        TBDG_AMR_T(3)
        TBDG_AMR_T(4)
        TBDG_AMR_T(5)
        TBDG_AMR_T(6)
        TBDG_AMR_T(7)
        TBDG_AMR_T(8)
        default: throw Error(TBDG_EUNSUPPORTED, "nodes per direction must be 1..8");
    }
#undef TBDG_AMR_T
    TBDG_HIP(hipGetLastError());
}

void launch_amr_dot(hipStream_t st, int64_t n, const double* a, const double* b, double* part, int G,
                    double* out) {
    hipLaunchKernelGGL(k_amr_dot, dim3(G), dim3(256), 0, st, n, a, b, part);
    hipLaunchKernelGGL(k_amr_dot_finish, dim3(1), dim3(256), 0, st, part, G, out);
    TBDG_HIP(hipGetLastError());
}

void launch_amr_maxdiff(hipStream_t st, int64_t n, const double* a, const double* b, double* part, int G,
                       double* out) {
    hipLaunchKernelGGL(k_amr_maxdiff, dim3(G), dim3(256), 0, st, n, a, b, part);
    hipLaunchKernelGGL(k_amr_max_finish, dim3(1), dim3(256), 0, st, part, G, out);
    TBDG_HIP(hipGetLastError());
}

bool amr_block_ok(int nb) { return nb == 1 || nb == 4 || nb == 9 || nb == 16; }

void launch_amr_block_build(hipStream_t st, const Geo& g, const Tab1& t, double alpha, double* u,
                            double* y, double* B, float* Binv) {
    const int nb = t.n * t.n;
    const int64_t nc = g.Nc;
    if (nc == 0) return;
    const int G = blocks(nc * nb);
    for (int i = 0; i < nb; ++i) {
        hipLaunchKernelGGL(k_amr_unit, dim3(G), dim3(256), 0, st, nc, nb, i, u);
        launch_amr_pressure_mode(st, g, t, alpha, u, y, 2, nullptr);
        hipLaunchKernelGGL(k_amr_block_col, dim3(G), dim3(256), 0, st, nc, nb, i, y, B);
    }
    const int Gi = (int)((nc + 63) / 64);
    switch (nb) {
        case 1: hipLaunchKernelGGL((k_amr_block_inv<1>), dim3(Gi), dim3(64), 0, st, nc, B, Binv); break;
        case 4: hipLaunchKernelGGL((k_amr_block_inv<4>), dim3(Gi), dim3(64), 0, st, nc, B, Binv); break;
        case 9: hipLaunchKernelGGL((k_amr_block_inv<9>), dim3(Gi), dim3(64), 0, st, nc, B, Binv); break;
        case 16: hipLaunchKernelGGL((k_amr_block_inv<16>), dim3(Gi), dim3(64), 0, st, nc, B, Binv); break;
        default: throw Error(TBDG_EUNSUPPORTED, "cell blocks up to 16 pressure nodes");
    }
    TBDG_HIP(hipGetLastError());
}

int amr_block_grid(int64_t nc, int nb) {
    const int cpb = 256 / nb;
    return (int)((nc + cpb - 1) / cpb);
}

namespace {

int block_apply(hipStream_t st, int64_t nc, int nb, const float* Binv, double* r, double* z, double* part,
                const CgUpdate* xr) {
    if (nc == 0) return 0;
    const int G = amr_block_grid(nc, nb);
    const CgUpdate u = xr ? *xr : CgUpdate{};
#define TBDG_AMR_B(NBV)                                                                       \
    case NBV:                                                                                 \
        if (xr) hipLaunchKernelGGL((k_amr_block_apply<NBV, true>), dim3(G), dim3(256), 0, st, nc, Binv, \
                                   r, z, part, u);                                           \
        else hipLaunchKernelGGL((k_amr_block_apply<NBV, false>), dim3(G), dim3(256), 0, st, nc, Binv, \
                                r, z, part, u);                                              \
        break;
    switch (nb) {
        TBDG_AMR_B(1)
        TBDG_AMR_B(4)
        TBDG_AMR_B(9)
        TBDG_AMR_B(16)
        default: throw Error(TBDG_EUNSUPPORTED, "cell blocks up to 16 pressure nodes");
    }
#undef TBDG_AMR_B
    TBDG_HIP(hipGetLastError());
    return G;
}

}  // namespace

int launch_amr_block_apply(hipStream_t st, int64_t nc, int nb, const float* Binv, const double* r,
                           double* z, double* part) {
    // without the update the kernel only reads r
    return block_apply(st, nc, nb, Binv, const_cast<double*>(r), z, part, nullptr);
}

int launch_amr_block_xr(hipStream_t st, int64_t nc, int nb, const float* Binv, const CgUpdate& xr,
                        double* r, double* z, double* part) {
    return block_apply(st, nc, nb, Binv, r, z, part, &xr);
}

void launch_amr_cg_step(hipStream_t st, int64_t n, const CgUpdate& u, const double* d, double* r,
                        double* z, double* part, int G) {
    hipLaunchKernelGGL(k_amr_cg_step, dim3(G), dim3(256), 0, st, n, u, d, r, z, part);
    TBDG_HIP(hipGetLastError());
}

void launch_amr_finish(hipStream_t st, const double* part, int G, int rows, double* out0, double* out1) {
    hipLaunchKernelGGL(k_amr_finish2, dim3(1), dim3(256), 0, st, part, G, rows, out0, out1);
    TBDG_HIP(hipGetLastError());
}

void launch_amr_div(hipStream_t st, int64_t n, const double* r, const double* d, double* z) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_amr_div, dim3(blocks(n)), dim3(256), 0, st, n, r, d, z);
    TBDG_HIP(hipGetLastError());
}

}  // namespace amr
}  // namespace trbdg
