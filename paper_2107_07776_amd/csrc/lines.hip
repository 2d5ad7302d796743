// Line-structured operator kernels for affine Cartesian boxes.
//
// With a Lagrange basis collocated at the Gauss points, the tangential mass
// of every volume and face integral is diagonal, so on a box with cell size
// h_a per direction every form of Sec. 3 splits into a sum over directions a
// of one-dimensional operators acting along the grid line through a node:
//
//   SIP (eq. bilin_diff, a_p):  sum_a |K|/h_a^2 * Wt_a(node) *
//                               [ A p(own line) + Lm p(left line) + Rm p(right line) ]
//   LF advection (eq. trilinear): sum_a |K|/h_a * Wt_a(node) *
//       [ -sum_m W_m u(m) w_a(m) l_i'(x_m) + l_i(0) F_left + l_i(1) F_right ]
//
// where A, Lm, Rm are the n x n element matrices of the 1D SIP form (cell
// stiffness plus the self and neighbour terms of the two end faces, reference
// cell of unit length), Wt_a is the product of the Gauss weights in the
// directions other than a, and F are the local Lax-Friedrichs fluxes at the
// two ends of the line.  Each thread owns one node and evaluates its row of
// every 1D operator directly: no face buffer, no block-wide exchange beyond
// the staging of its own cell.
#include "internal.hpp"
#include "lines.hpp"
#include "reduce.hpp"

#include <hip/hip_ext.h>

namespace trbdg {
namespace {

using namespace lines;

// ============================================================================
// Pressure Helmholtz operator y = alpha M^p p + K p
// ============================================================================
// MODE 0: y = H p; MODE 1: y = diag(H); MODE 2: y = H p and, fused, one
// partial sum of p . y per block (the CG step length is formed by a separate
// one-block kernel: a grid-wide fence per block costs more than a launch on
// a multi-XCD device).
template <int DIM, int NP, int MODE>
__global__ __launch_bounds__(256) void k_pressure_line(Geom g, LineGeom lg, Line1D lt, Tables t,
                                                        double cm, const double* __restrict__ p,
                                                        double* __restrict__ y, int Nc,
                                                        double* partial) {
    using L = Lay<DIM, NP>;
    constexpr int NB = L::NB;
    constexpr int NN = NP * NP;
    constexpr bool DIAG = MODE == 1;
    // the 1D element matrices are indexed by the thread's own node: stage
    // them in LDS rather than gathering from the kernel-argument segment
    __shared__ double s_m[5 * NN + NP];
    for (int i = threadIdx.x; i < 5 * NN + NP; i += blockDim.x) {
        const int mtx = i / NN, e = i % NN;
        s_m[i] = mtx == 0 ? lt.A[e] : mtx == 1 ? lt.F0[e] : mtx == 2 ? lt.F1[e] : mtx == 3 ? lt.Lm[e]
               : mtx == 4 ? lt.Rm[e] : t.Wp[e];
    }
    __syncthreads();
    const double* Wp = s_m + 5 * NN;
    const double* A = s_m;
    const double* F0 = s_m + NN;
    const double* F1 = s_m + 2 * NN;
    const double* Lm = s_m + 3 * NN;
    const double* Rm = s_m + 4 * NN;
    const int gid = blockIdx.x * 256 + threadIdx.x;
    if (MODE != 2 && gid >= Nc * NB) return;
    const bool active = gid < Nc * NB;
    const int cell = active ? gid / NB : 0, nd = active ? gid % NB : 0;
    const Nbrs<DIM> nb(g, lg, cell);
    double acc = cm * L::wnode(Wp, nd) * (DIAG ? 1.0 : (active ? p[gid] : 0.0));
    for (int a = 0; a < DIM; ++a) {
        const int ia = L::coord(nd, a), tt = L::tang(nd, a);
        const int lf = nb.left[a], rt = nb.right[a];
        double s = 0.0;
        if (!active) {
        } else if (DIAG) {
            s = A[ia * NP + ia];
            if (lf < 0) s += lg.wall * F0[ia * NP + ia];
            if (rt < 0) s += lg.wall * F1[ia * NP + ia];
            if (lf == cell) s += Lm[ia * NP + ia];
            if (rt == cell) s += Rm[ia * NP + ia];
        } else {
#pragma unroll
            for (int j = 0; j < NP; ++j) {
                const int idx = L::node(a, j, tt);
                double c = A[ia * NP + j];
                if (lf < 0) c += lg.wall * F0[ia * NP + j];
                if (rt < 0) c += lg.wall * F1[ia * NP + j];
                s += c * p[cell * NB + idx];
                if (lf >= 0) s += Lm[ia * NP + j] * p[lf * NB + idx];
                if (rt >= 0) s += Rm[ia * NP + j] * p[rt * NB + idx];
            }
        }
        acc += lg.sdiff[a] * L::wtan(Wp, tt) * s;
    }
    if (active) y[gid] = acc;
    if (MODE == 2) {
        const double pq = red::block_sum(active ? acc * p[gid] : 0.0);
        if (threadIdx.x == 0) partial[blockIdx.x] = pq;
    }
}

// ============================================================================
// Momentum operator y_c = m M u_c + theta (nu A u_c + C(w) u_c), all c
// ============================================================================
template <int DIM, int N, bool DIAG>
__global__ __launch_bounds__(256) void k_momentum_line(Geom g, LineGeom lg, Line1D lt, Tables t,
                                                        double mc, double tnu, double th,
                                                        const double* __restrict__ w,
                                                        const double* __restrict__ u,
                                                        double* __restrict__ y, int Nc, Bnd bd) {
    using L = Lay<DIM, N>;
    constexpr int NB = L::NB, CPB = L::CPB;
    __shared__ double s_w[DIM][CPB * NB];
    __shared__ double s_u[DIM][CPB * NB];
    constexpr int NN = N * N;
    __shared__ double s_m[6 * NN + 3 * N];
    for (int i = threadIdx.x; i < 6 * NN + 3 * N; i += blockDim.x) {
        double v;
        if (i < 5 * NN) {
            const int mtx = i / NN, e = i % NN;
            v = mtx == 0 ? lt.A[e] : mtx == 1 ? lt.F0[e] : mtx == 2 ? lt.F1[e] : mtx == 3 ? lt.Lm[e] : lt.Rm[e];
        } else if (i < 6 * NN) {
            v = t.Du[i - 5 * NN];
        } else {
            const int e = i - 6 * NN;
            v = e < N ? t.Wu[e] : (e < 2 * N ? t.L0u[e - N] : t.L1u[e - 2 * N]);
        }
        s_m[i] = v;
    }
    const double* mA = s_m;
    const double* mF0 = s_m + NN;
    const double* mF1 = s_m + 2 * NN;
    const double* mLm = s_m + 3 * NN;
    const double* mRm = s_m + 4 * NN;
    const double* D = s_m + 5 * NN;
    const double* Wv = s_m + 6 * NN;
    const double* L0v = Wv + N;
    const double* L1v = Wv + 2 * N;
    const int tid = threadIdx.x;
    const int lc = tid / NB, nd = tid % NB;
    const int cell = blockIdx.x * CPB + lc;
    const bool active = cell < Nc;
    for (int c = 0; c < DIM; ++c) {
        s_w[c][tid] = active ? w[((size_t)cell * DIM + c) * NB + nd] : 0.0;
        if (!DIAG) s_u[c][tid] = active ? u[((size_t)cell * DIM + c) * NB + nd] : 0.0;
    }
    __syncthreads();
    if (!active) return;
    const Nbrs<DIM> nb(g, lg, cell);
    const double Wi = L::wnode(Wv, nd);
    double acc[DIM];
    for (int c = 0; c < DIM; ++c) acc[c] = mc * Wi * (DIAG ? 1.0 : s_u[c][tid]);
    const int base = lc * NB;
    for (int a = 0; a < DIM; ++a) {
        const int ia = L::coord(nd, a), tt = L::tang(nd, a);
        const int lf = nb.left[a], rt = nb.right[a];
        const double wt = L::wtan(Wv, tt);
        // traces of the advecting component w_a at both ends of the line
        double w0 = 0.0, w1 = 0.0, wl = 0.0, wr = 0.0;
        double wline[N];
#pragma unroll
        for (int m = 0; m < N; ++m) {
            const int idx = L::node(a, m, tt);
            const double wo = s_w[a][base + idx];
            wline[m] = wo;
            w0 += t.L0u[m] * wo;
            w1 += t.L1u[m] * wo;
            if (lf >= 0) wl += t.L1u[m] * w[((size_t)lf * DIM + a) * NB + idx];
            if (rt >= 0) wr += t.L0u[m] * w[((size_t)rt * DIM + a) * NB + idx];
        }
        const double lam0 = fmax(fabs(w0), fabs(wl));
        const double lam1 = fmax(fabs(w1), fabs(wr));
        const double sd = tnu * lg.sdiff[a] * wt;
        const double sv = th * lg.sadv[a] * wt;
        if (DIAG) {
            // Dirichlet faces (no neighbour): the self term once more, and
            // lambda u v with lambda from the mirrored state 2 u_D - w
            double s = mA[ia * N + ia];
            if (lf < 0) s += mF0[ia * N + ia];
            if (rt < 0) s += mF1[ia * N + ia];
            if (lf == cell) s += mLm[ia * N + ia];
            if (rt == cell) s += mRm[ia * N + ia];
            const double L0 = L0v[ia], L1 = L1v[ia];
            double v = -Wv[ia] * wline[ia] * D[ia * N + ia];
            if (lf >= 0) v += L0 * L0 * 0.5 * (-w0 + lam0);
            if (rt >= 0) v += L1 * L1 * 0.5 * (w1 + lam1);
            if (lf < 0) {
                const double uDa = bd.uD[bnd_point(bd, g, cell, a, 0, tt, L::NB / N) * DIM + a];
                v += L0 * L0 * fmax(fabs(w0), fabs(2.0 * uDa - w0));
            }
            if (rt < 0) {
                const double uDa = bd.uD[bnd_point(bd, g, cell, a, 1, tt, L::NB / N) * DIM + a];
                v += L1 * L1 * fmax(fabs(w1), fabs(2.0 * uDa - w1));
            }
            if (lf == cell) v += L0 * L1 * 0.5 * (-wl - lam0);
            if (rt == cell) v += L1 * L0 * 0.5 * (wr - lam1);
            acc[0] += sd * s + sv * v;
            continue;
        }
        for (int c = 0; c < DIM; ++c) {
            double s = 0.0, vol = 0.0;
            double u0 = 0.0, u1 = 0.0, ul = 0.0, ur = 0.0;
#pragma unroll
            for (int j = 0; j < N; ++j) {
                const int idx = L::node(a, j, tt);
                const double uo = s_u[c][base + idx];
                double cf = mA[ia * N + j];
                if (lf < 0) cf -= mF0[ia * N + j];
                if (rt < 0) cf -= mF1[ia * N + j];
                s += cf * uo;
                u0 += t.L0u[j] * uo;
                u1 += t.L1u[j] * uo;
                vol -= t.Wu[j] * uo * wline[j] * D[j * N + ia];
                if (lf >= 0) {
                    const double ulv = u[((size_t)lf * DIM + c) * NB + idx];
                    s += mLm[ia * N + j] * ulv;
                    ul += t.L1u[j] * ulv;
                }
                if (rt >= 0) {
                    const double urv = u[((size_t)rt * DIM + c) * NB + idx];
                    s += mRm[ia * N + j] * urv;
                    ur += t.L0u[j] * urv;
                }
            }
            double fl = 0.0, fr = 0.0;
            if (lf >= 0) fl = 0.5 * (-u0 * w0 - ul * wl) + 0.5 * lam0 * (u0 - ul);
            if (rt >= 0) fr = 0.5 * (u1 * w1 + ur * wr) + 0.5 * lam1 * (u1 - ur);
            acc[c] += sd * s + sv * (vol + L0v[ia] * fl + L1v[ia] * fr);
        }
    }
    if (DIAG) {
        y[(size_t)cell * NB + nd] = acc[0];
    } else {
        for (int c = 0; c < DIM; ++c) y[((size_t)cell * DIM + c) * NB + nd] = acc[c];
    }
}

// ============================================================================
// Operator kernels (apply).  Three phases per block of CPB whole cells:
//  1. stage the own cells in LDS and gather, for every face point of every
//     own cell, the neighbour's trace value v and normal derivative d (the
//     neighbour enters each 1D SIP coupling only through them:
//       sum_j Lm[i][j] u_left(j) = l_i(0) (d_L/2 - Cr v_L) - l_i'(0) v_L/2,
//     and symmetrically on the right) and, for the momentum operator, the
//     neighbour's advecting-velocity trace;
//  2. one work item per (cell, direction, [component,] grid line) applies the
//     1D operators of that line to its n nodes with all per-line quantities
//     (end traces, LF fluxes, the u w products) computed once, and stores the
//     n results per direction in LDS;
//  3. one thread per node adds the mass term and the directions and writes.
// Blocks are mapped to cells XCD by XCD (the hardware hands consecutive
// blocks to the 8 XCDs in turn), so each XCD sweeps a contiguous slab of
// cells and the neighbour lines it gathers mostly hit its own L2.
// ============================================================================

template <int DIM, int N>
__global__ __launch_bounds__(256) void k_momentum_face(Geom g, LineGeom lg, Line1D lt, Tables t,
                                                        double Cr, double mc, double tnu, double th,
                                                        const double* __restrict__ w,
                                                        const double* __restrict__ u,
                                                        double* __restrict__ y, int Nc, Bnd bd,
                                                        MomFuse fz, int zc) {
    using L = Lay<DIM, N>;
    using F = FaceLay<DIM, N>;
    constexpr int NB = F::NB, NF = F::NF, CPB = F::CPB;
    constexpr int REC = 2 * DIM + 1;
    const double us = fz.invd ? fz.gsc[0] : 1.0;
    double uraw[DIM];
#pragma unroll
    for (int c = 0; c < DIM; ++c) uraw[c] = 0.0;
    // per-cell node arrays padded by one slot per x-row: lanes walking
    // x-lines then touch distinct LDS banks
    constexpr int NBP = NB + NB / N;
    __shared__ double s_wa[CPB * NBP];
    __shared__ double s_u[DIM][CPB * NBP];
    __shared__ double s_y[DIM][CPB * NBP];
    __shared__ double s_f[CPB * 2 * NF * REC];   // face records of one direction
    __shared__ int s_nbr[CPB * 2 * DIM];
    __shared__ int s_cell[CPB];
    __shared__ double s_W[N];
    const int tid = threadIdx.x;
    if (tid < N) s_W[tid] = t.Wu[tid];
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    const int lc = tid / NB, nd = tid % NB;
    const int cell = lc < CPB ? tile_cell(blk, lc, g, CPB, zc, Nc) : -1;
    const bool active = cell >= 0;
    const int pi = lc * NBP + nd + nd / N;
    double wreg[DIM];
    if (lc < CPB) {
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            s_u[c][pi] = active ? u[((size_t)cell * DIM + c) * NB + nd] : 0.0;
            wreg[c] = active ? w[((size_t)cell * DIM + c) * NB + nd] : 0.0;
        }
        if (fz.invd && active) {
            const double sc = us * fz.invd[(size_t)cell * NB + nd];
#pragma unroll
            for (int c = 0; c < DIM; ++c) {
                uraw[c] = s_u[c][pi];
                s_u[c][pi] *= sc;
            }
        }
    }
    if (lc < CPB && nd == 0) {
        s_cell[lc] = cell;
        // neighbour table of the cell, written with constant indices
        const Nbrs<DIM> nb(g, lg, active ? cell : 0);
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            s_nbr[lc * 2 * DIM + 2 * a] = active ? nb.left[a] : -1;
            s_nbr[lc * 2 * DIM + 2 * a + 1] = active ? nb.right[a] : -1;
        }
    }
    __syncthreads();
    // phase 2 (with phase 1 per direction): one pass per direction, items
    // (cell, component, line); each node receives exactly one contribution
    // per pass
    if (lc < CPB) {
        const double Wi0 = L::wnode(s_W, nd);
#pragma unroll
        for (int c = 0; c < DIM; ++c) s_y[c][pi] = mc * Wi0 * s_u[c][pi];
    }
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        if (lc < CPB) s_wa[pi] = wreg[a];
        // phase 1 for direction a: the two faces of every own cell
        for (int it = tid; it < CPB * 2 * NF; it += 256) {
            const int lc1 = it / (2 * NF), s = (it / NF) & 1, tt = it % NF;
            double rec[REC];
#pragma unroll
            for (int q = 0; q < REC; ++q) rec[q] = 0.0;
            const int nbr = s_nbr[lc1 * 2 * DIM + 2 * a + s];
            if (nbr >= 0) {
#pragma unroll
                for (int m = 0; m < N; ++m) {
                    const int idx = L::node(a, m, tt);
                    const double lo = s ? t.L0u[m] : t.L1u[m];
                    const double dlo = s ? t.dL0u[m] : t.dL1u[m];
                    rec[2 * DIM] += lo * w[((size_t)nbr * DIM + a) * NB + idx];
                    const double sc = fz.invd ? us * fz.invd[(size_t)nbr * NB + idx] : 1.0;
#pragma unroll
                    for (int c = 0; c < DIM; ++c) {
                        const double uv = sc * u[((size_t)nbr * DIM + c) * NB + idx];
                        rec[2 * c] += lo * uv;
                        rec[2 * c + 1] += dlo * uv;
                    }
                }
            }
            double* dst = s_f + it * REC;
#pragma unroll
            for (int q = 0; q < REC; ++q) dst[q] = rec[q];
        }
        __syncthreads();
        constexpr int ITEMS = CPB * DIM * NF;
        for (int it = tid; it < ITEMS; it += 256) {
            const int lc2 = it / (DIM * NF);
            const int c = (it % (DIM * NF)) / NF, ln = it % NF;
            const int cell2 = s_cell[lc2];
            if (cell2 < 0) continue;
            const int base = lc2 * NBP;
            double uu[N], uw[N];
            double u0 = 0.0, u1 = 0.0, w0 = 0.0, w1 = 0.0, q0 = 0.0, q1 = 0.0;
#pragma unroll
            for (int m = 0; m < N; ++m) {
                const int nm = L::node(a, m, ln);
                const int idx = base + nm + nm / N;
                const double um = s_u[c][idx], wm = s_wa[idx];
                uu[m] = um;
                uw[m] = um * wm;
                u0 += t.L0u[m] * um;
                u1 += t.L1u[m] * um;
                w0 += t.L0u[m] * wm;
                w1 += t.L1u[m] * wm;
            }
            const double* recl = s_f + ((lc2 * 2) * NF + ln) * REC;
            const double* recr = s_f + ((lc2 * 2 + 1) * NF + ln) * REC;
            const bool hl = s_nbr[lc2 * 2 * DIM + 2 * a] >= 0;
            const bool hr = s_nbr[lc2 * 2 * DIM + 2 * a + 1] >= 0;
            double X0, Y0, X1, Y1, fl = 0.0, fr = 0.0;
            if (hl) {
                const double vL = recl[2 * c], dL = recl[2 * c + 1], wl = recl[2 * DIM];
                const double lam = fmax(fabs(w0), fabs(wl));
                X0 = 0.5 * dL - Cr * vL;
                Y0 = 0.5 * vL;
                fl = 0.5 * (-u0 * w0 - vL * wl) + 0.5 * lam * (u0 - vL);
            } else {
                // Dirichlet face: SIP terms with twice the penalty (the self
                // term once more) and the LF term lambda u v, lambda from the
                // mirrored state 2 u_D - w
#pragma unroll
                for (int m = 0; m < N; ++m) q0 += t.dL0u[m] * uu[m];
                X0 = 0.5 * q0 + Cr * u0;
                Y0 = -0.5 * u0;
                const double uDa = bd.uD[bnd_point(bd, g, cell2, a, 0, ln, NF) * DIM + a];
                fl = fmax(fabs(w0), fabs(2.0 * uDa - w0)) * u0;
            }
            if (hr) {
                const double vR = recr[2 * c], dR = recr[2 * c + 1], wr = recr[2 * DIM];
                const double lam = fmax(fabs(w1), fabs(wr));
                X1 = -0.5 * dR - Cr * vR;
                Y1 = 0.5 * vR;
                fr = 0.5 * (u1 * w1 + vR * wr) + 0.5 * lam * (u1 - vR);
            } else {
#pragma unroll
                for (int m = 0; m < N; ++m) q1 += t.dL1u[m] * uu[m];
                X1 = -0.5 * q1 + Cr * u1;
                Y1 = -0.5 * u1;
                const double uDa = bd.uD[bnd_point(bd, g, cell2, a, 1, ln, NF) * DIM + a];
                fr = fmax(fabs(w1), fabs(2.0 * uDa - w1)) * u1;
            }
            const double wt = L::wtan(s_W, ln);
            const double sd = tnu * lg.sdiff[a] * wt;
            const double sv = th * lg.sadv[a] * wt;
            const double cl = sd * X0 + sv * fl, cr = sd * X1 + sv * fr;
            const double dl = sd * Y0, dr = sd * Y1;
#pragma unroll
            for (int i = 0; i < N; ++i) {
                double s = 0.0, vol = 0.0;
#pragma unroll
                for (int j = 0; j < N; ++j) {
                    s += lt.A[i * N + j] * uu[j];
                    vol -= lt.WD[j * N + i] * uw[j];
                }
                const double out = sd * s + sv * vol + t.L0u[i] * cl + t.L1u[i] * cr
                                   - t.dL0u[i] * dl + t.dL1u[i] * dr;
                const int ni = L::node(a, i, ln);
                s_y[c][base + ni + ni / N] += out;
            }
        }
        // the next direction's gathers overwrite s_f and its items touch
        // other nodes of s_y
        __syncthreads();
    }
    double yv[DIM];
    const double ysh = fz.invd ? fz.shift * us : (fz.shv ? fz.shift * fz.gsc[0] : 0.0);
    if (fz.shv && active) {
#pragma unroll
        for (int c = 0; c < DIM; ++c) uraw[c] = fz.shv[((size_t)cell * DIM + c) * NB + nd];
    }
#pragma unroll
    for (int c = 0; c < DIM; ++c) yv[c] = active ? s_y[c][pi] - ysh * uraw[c] : 0.0;
    if (fz.rb && active) {
#pragma unroll
        for (int c = 0; c < DIM; ++c) yv[c] = fz.rb[((size_t)cell * DIM + c) * NB + nd] - yv[c];
    }
    if (active) {
#pragma unroll
        for (int c = 0; c < DIM; ++c) y[((size_t)cell * DIM + c) * NB + nd] = yv[c];
    }
    if (fz.ndot > 0) {
        // partial sums of y . V_i and y . y over the block's nodes: one wave
        // sum per value, then one thread per value adds the four waves
        __shared__ double s_red[MOM_FUSE_MAX_DOTS + 1][4];
        const int lane = tid & 63, wv = tid >> 6;
#pragma unroll
        for (int i = 0; i <= MOM_FUSE_MAX_DOTS; ++i) {
            if (i > fz.ndot) break;
            double v = 0.0;
            if (active) {
#pragma unroll
                for (int c = 0; c < DIM; ++c) {
                    const size_t gi = ((size_t)cell * DIM + c) * NB + nd;
                    v += yv[c] * (i < fz.ndot ? fz.V[(size_t)i * fz.ldv + gi] : yv[c]);
                }
            }
            v = red::wave_sum(v);
            if (lane == 0) s_red[i][wv] = v;
        }
        __syncthreads();
        if (tid <= fz.ndot) {
            const double r = s_red[tid][0] + s_red[tid][1] + s_red[tid][2] + s_red[tid][3];
            fz.part[(size_t)tid * gridDim.x + blockIdx.x] = r;
        }
    }
}

// Line-block preconditioner of the momentum operator (not in the paper, which
// uses Jacobi): P^{-1} = B_z^{-1} D B_y^{-1} D B_x^{-1} (2D: B_y^{-1} D B_x^{-1}),
// B_a = the exact restriction of the scalar stage operator to each grid line
// of direction a inside a cell: the full Jacobi diagonal D on its diagonal
// and the couplings of direction a's line operator (stiffness, advection
// volume term, the own-trace parts of the SIP and Lax-Friedrichs face terms,
// Dirichlet self terms) off it.  The same for every velocity component.
//
// Set-up: one thread per (cell, direction, line) assembles B_a in FP64 and
// stores its inverse (Gauss-Jordan with partial pivoting) rounded to FP32 at
// blk[((a Nc + cell) NF + line) N^2 + i N + j]; the apply computes in FP64
// with these fixed coefficients, so P^{-1} stays one linear operator.
template <int DIM, int N>
__global__ __launch_bounds__(256) void k_mom_lineblk(Geom g, LineGeom lg, Line1D lt, Tables t,
                                                      double Cr, double tnu, double th,
                                                      const double* __restrict__ w,
                                                      const double* __restrict__ d,
                                                      float* __restrict__ blk, int Nc, Bnd bd) {
    using L = Lay<DIM, N>;
    constexpr int NB = L::NB;
    constexpr int NF = ipow(N, DIM - 1);
    const int64_t it = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (it >= (int64_t)Nc * DIM * NF) return;
    const int ln = (int)(it % NF);
    const int a = (int)((it / NF) % DIM);
    const int cell = (int)(it / ((int64_t)DIM * NF));
    const Nbrs<DIM> nb(g, lg, cell);
    int left = nb.left[0], right = nb.right[0];
#pragma unroll
    for (int e = 1; e < DIM; ++e)
        if (a == e) {
            left = nb.left[e];
            right = nb.right[e];
        }
    double wl[N], dd[N];
    double w0 = 0.0, w1 = 0.0, wL = 0.0, wR = 0.0;
#pragma unroll
    for (int m = 0; m < N; ++m) {
        const int nm = L::node(a, m, ln);
        wl[m] = w[((size_t)cell * DIM + a) * NB + nm];
        dd[m] = d[(size_t)cell * NB + nm];
        w0 += t.L0u[m] * wl[m];
        w1 += t.L1u[m] * wl[m];
        if (left >= 0) wL += t.L1u[m] * w[((size_t)left * DIM + a) * NB + nm];
        if (right >= 0) wR += t.L0u[m] * w[((size_t)right * DIM + a) * NB + nm];
    }
    const double wt = L::wtan(t.Wu, ln);
    const double sd = tnu * lg.sdiff[a] * wt, sv = th * lg.sadv[a] * wt;
    // own-trace derivatives of the face terms: cl = sd X0 + sv fl and dl = sd Y0
    // on the left face (coefficients of L0_j and dL0_j), the same on the right
    double cl_v, cl_d, dl_v, cr_v, cr_d, dr_v;
    if (left >= 0) {
        const double lam = fmax(fabs(w0), fabs(wL));
        cl_v = sv * 0.5 * (lam - w0);
        cl_d = 0.0;
        dl_v = 0.0;
    } else {
        const double uDa = bd.uD[bnd_point(bd, g, cell, a, 0, ln, NF) * DIM + a];
        const double lam = fmax(fabs(w0), fabs(2.0 * uDa - w0));
        cl_v = sd * Cr + sv * lam;
        cl_d = sd * 0.5;
        dl_v = -sd * 0.5;
    }
    if (right >= 0) {
        const double lam = fmax(fabs(w1), fabs(wR));
        cr_v = sv * 0.5 * (lam + w1);
        cr_d = 0.0;
        dr_v = 0.0;
    } else {
        const double uDa = bd.uD[bnd_point(bd, g, cell, a, 1, ln, NF) * DIM + a];
        const double lam = fmax(fabs(w1), fabs(2.0 * uDa - w1));
        cr_v = sd * Cr + sv * lam;
        cr_d = -sd * 0.5;
        dr_v = -sd * 0.5;
    }
    double B[N][2 * N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
#pragma unroll
        for (int j = 0; j < N; ++j) {
            // left face: L0_i (cl_v L0_j + cl_d dL0_j) - dL0_i dl_v L0_j;
            // right face: L1_i (cr_v L1_j + cr_d dL1_j) + dL1_i dr_v L1_j
            const double v = sd * lt.A[i * N + j] - sv * lt.WD[j * N + i] * wl[j] +
                             t.L0u[i] * (cl_v * t.L0u[j] + cl_d * t.dL0u[j]) -
                             t.dL0u[i] * dl_v * t.L0u[j] +
                             t.L1u[i] * (cr_v * t.L1u[j] + cr_d * t.dL1u[j]) +
                             t.dL1u[i] * dr_v * t.L1u[j];
            B[i][j] = i == j ? dd[i] : v;
            B[i][N + j] = i == j ? 1.0 : 0.0;
        }
    }
    // Gauss-Jordan with partial pivoting (rows swapped by value)
#pragma unroll
    for (int k = 0; k < N; ++k) {
        int piv = k;
        double best = fabs(B[k][k]);
#pragma unroll
        for (int r = k + 1; r < N; ++r)
            if (fabs(B[r][k]) > best) {
                best = fabs(B[r][k]);
                piv = r;
            }
#pragma unroll
        for (int r = k + 1; r < N; ++r) {
            if (r != piv) continue;
#pragma unroll
            for (int q = 0; q < 2 * N; ++q) {
                const double tmp = B[k][q];
                B[k][q] = B[r][q];
                B[r][q] = tmp;
            }
        }
        const double inv = 1.0 / B[k][k];
#pragma unroll
        for (int q = 0; q < 2 * N; ++q) B[k][q] *= inv;
#pragma unroll
        for (int r = 0; r < N; ++r) {
            if (r == k) continue;
            const double f = B[r][k];
#pragma unroll
            for (int q = 0; q < 2 * N; ++q) B[r][q] -= f * B[k][q];
        }
    }
    float* out = blk + ((size_t)((int64_t)a * Nc + cell) * NF + ln) * (N * N);
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int j = 0; j < N; ++j) out[i * N + j] = (float)B[i][N + j];
}

// Apply: z = P^{-1} (s v), s = *scale (1 when scale is null), per velocity
// component; the own cells staged in LDS, one pass per direction, one work
// item per (cell, component, line) with the line fastest (consecutive lanes
// read consecutive blocks, and their LDS accesses fall on distinct banks:
// with the component fastest, the three components of a node share a bank),
// scaled by D between the passes.
template <int DIM, int N>
__global__ __launch_bounds__(256) void k_mom_lineprec(const float* __restrict__ blk,
                                                       const double* __restrict__ d,
                                                       const double* __restrict__ v,
                                                       const double* __restrict__ scale,
                                                       double* __restrict__ z, int Nc, int acc) {
    using L = Lay<DIM, N>;
    using F = FaceLay<DIM, N>;
    constexpr int NB = F::NB, NF = F::NF, CPB = F::CPB;
    constexpr int NBP = NB + NB / N;
    __shared__ double s_v[DIM][CPB * NBP];
    const int tid = threadIdx.x;
    const int lc = tid / NB, nd = tid % NB;
    const int cell = blockIdx.x * CPB + lc;
    const bool active = lc < CPB && cell < Nc;
    const int pi = lc * NBP + nd + nd / N;
    const double sc = scale ? scale[0] : 1.0;
    double dn = 0.0;
    if (lc < CPB) {
        dn = active ? d[(size_t)cell * NB + nd] : 0.0;
#pragma unroll
        for (int c = 0; c < DIM; ++c)
            s_v[c][pi] = active ? sc * v[((size_t)cell * DIM + c) * NB + nd] : 0.0;
    }
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        __syncthreads();
        constexpr int ITEMS = CPB * DIM * NF;
        for (int it = tid; it < ITEMS; it += 256) {
            const int lc2 = it / (DIM * NF);
            const int c = (it % (DIM * NF)) / NF, ln = it % NF;
            const int cell2 = blockIdx.x * CPB + lc2;
            if (cell2 >= Nc) continue;
            const float* Bi = blk + ((size_t)((int64_t)a * Nc + cell2) * NF + ln) * (N * N);
            double x[N];
#pragma unroll
            for (int m = 0; m < N; ++m) {
                const int nm = L::node(a, m, ln);
                x[m] = s_v[c][lc2 * NBP + nm + nm / N];
            }
#pragma unroll
            for (int i = 0; i < N; ++i) {
                double acc = 0.0;
#pragma unroll
                for (int j = 0; j < N; ++j) acc += (double)Bi[i * N + j] * x[j];
                const int nm = L::node(a, i, ln);
                s_v[c][lc2 * NBP + nm + nm / N] = acc;
            }
        }
        __syncthreads();
        if (a + 1 < DIM && lc < CPB) {
#pragma unroll
            for (int c = 0; c < DIM; ++c) s_v[c][pi] *= dn;
        }
    }
    if (active) {
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            const size_t gi = ((size_t)cell * DIM + c) * NB + nd;
            z[gi] = acc ? z[gi] + s_v[c][pi] : s_v[c][pi];
        }
    }
}

// Momentum right-hand side in line form (the functionals of eq. rhs1 and its
// stage-2 analogue):
//   rhs_c = m |K| W_i u_prev,c + sum_pairs [ -cd L0(u) + ca A0_w(u) ]_c + (Gw p)_c
// with, along direction a and per line (reference coordinate, h_a the cell
// size, wt the tangential weights, l0/l1 the nodal basis at the line ends):
//   L0: sdiff wt [ sum_j WD_ji (D u)_j - 1/2 (q1 + dR) l1_i + 1/2 (q0 + dL) l0_i ]
//   A0: sadv wt [ sum_j WD_ji (u w_a)_j - 1/2 (u1 w1 + vR wR) l1_i
//                 + 1/2 (u0 w0 + vL wL) l0_i ]
//   Gw (only a = c): sadv wt [ sum_j WD_ji p_j - 1/2 (p1 + pR) l1_i + 1/2 (p0 + pL) l0_i ]
// (u0, u1 the own end values, q0, q1 the own end derivatives, vL/vR, dL/dR,
// wL/wR, pL/pR the neighbour's; on a boundary face the average is the own
// trace).  The pressure enters through its interpolant pv at the velocity
// nodes.  Same block structure as the operator kernel: the own cells in LDS,
// one direction's neighbour records at a time, one work item per
// (cell, component, line).
template <int DIM, int N>
__global__ __launch_bounds__(256) void k_rhs_lines(Geom g, LineGeom lg, Line1D lt, Tables t,
                                                    double mcv, const double* __restrict__ uprev,
                                                    const double* __restrict__ u1,
                                                    const double* __restrict__ w1, double cd1,
                                                    double ca1, const double* __restrict__ u2,
                                                    const double* __restrict__ w2, double cd2,
                                                    double ca2, const double* __restrict__ pv,
                                                    double* __restrict__ rhs, int Nc) {
    using L = Lay<DIM, N>;
    using F = FaceLay<DIM, N>;
    constexpr int NB = F::NB, NF = F::NF, CPB = F::CPB;
    constexpr int REC = 2 * DIM + 2;
    constexpr int NBP = NB + NB / N;
    __shared__ double s_u[DIM][CPB * NBP];
    __shared__ double s_y[DIM][CPB * NBP];
    __shared__ double s_wa[CPB * NBP];
    __shared__ double s_p[CPB * NBP];
    __shared__ double s_f[CPB * 2 * NF * REC];
    __shared__ int s_nbr[CPB * 2 * DIM];
    __shared__ double s_W[N];
    const int tid = threadIdx.x;
    if (tid < N) s_W[tid] = t.Wu[tid];
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    const int lc = tid / NB, nd = tid % NB;
    const int cell = blk * CPB + lc;
    const bool active = lc < CPB && cell < Nc;
    const int pi = lc * NBP + nd + nd / N;
    if (lc < CPB) s_p[pi] = active ? pv[(size_t)cell * NB + nd] : 0.0;
    if (lc < CPB && nd == 0) {
        const Nbrs<DIM> nb(g, lg, active ? cell : 0);
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            s_nbr[lc * 2 * DIM + 2 * a] = active ? nb.left[a] : -1;
            s_nbr[lc * 2 * DIM + 2 * a + 1] = active ? nb.right[a] : -1;
        }
    }
    __syncthreads();
    if (lc < CPB) {
        const double Wi0 = L::wnode(s_W, nd);
#pragma unroll
        for (int c = 0; c < DIM; ++c)
            s_y[c][pi] = active ? mcv * Wi0 * uprev[((size_t)cell * DIM + c) * NB + nd] : 0.0;
    }
    const int npairs = u2 ? 2 : 1;
    for (int pr = 0; pr < npairs; ++pr) {
        const double* U = pr ? u2 : u1;
        const double* Wv = pr ? w2 : w1;
        const double cd = pr ? cd2 : cd1, ca = pr ? ca2 : ca1;
        const bool with_p = pr == 0;
        if (lc < CPB) {
#pragma unroll
            for (int c = 0; c < DIM; ++c)
                s_u[c][pi] = active ? U[((size_t)cell * DIM + c) * NB + nd] : 0.0;
        }
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            if (lc < CPB) s_wa[pi] = active ? Wv[((size_t)cell * DIM + a) * NB + nd] : 0.0;
            for (int it = tid; it < CPB * 2 * NF; it += 256) {
                const int lc1 = it / (2 * NF), sd = (it / NF) & 1, tt = it % NF;
                double rec[REC];
#pragma unroll
                for (int q = 0; q < REC; ++q) rec[q] = 0.0;
                const int nbr = s_nbr[lc1 * 2 * DIM + 2 * a + sd];
                if (nbr >= 0) {
#pragma unroll
                    for (int m = 0; m < N; ++m) {
                        const int idx = L::node(a, m, tt);
                        const double lo = sd ? t.L0u[m] : t.L1u[m];
                        const double dlo = sd ? t.dL0u[m] : t.dL1u[m];
                        rec[2 * DIM] += lo * Wv[((size_t)nbr * DIM + a) * NB + idx];
                        if (with_p) rec[2 * DIM + 1] += lo * pv[(size_t)nbr * NB + idx];
#pragma unroll
                        for (int c = 0; c < DIM; ++c) {
                            const double uv = U[((size_t)nbr * DIM + c) * NB + idx];
                            rec[2 * c] += lo * uv;
                            rec[2 * c + 1] += dlo * uv;
                        }
                    }
                }
                double* dst = s_f + it * REC;
#pragma unroll
                for (int q = 0; q < REC; ++q) dst[q] = rec[q];
            }
            __syncthreads();
            constexpr int ITEMS = CPB * DIM * NF;
            for (int it = tid; it < ITEMS; it += 256) {
                const int lc2 = it / (DIM * NF);
                const int c = (it % (DIM * NF)) / NF, ln = it % NF;
                if (blk * CPB + lc2 >= Nc) continue;
                const int base = lc2 * NBP;
                const bool pl = with_p && c == a;
                double uu[N], uw[N], pp[N];
                double u0 = 0.0, u1v = 0.0, w0 = 0.0, w1v = 0.0, q0 = 0.0, q1 = 0.0, p0 = 0.0, p1 = 0.0;
#pragma unroll
                for (int m = 0; m < N; ++m) {
                    const int nm = L::node(a, m, ln);
                    const int idx = base + nm + nm / N;
                    const double um = s_u[c][idx], wm = s_wa[idx];
                    uu[m] = um;
                    uw[m] = um * wm;
                    pp[m] = pl ? s_p[idx] : 0.0;
                    u0 += t.L0u[m] * um;
                    u1v += t.L1u[m] * um;
                    q0 += t.dL0u[m] * um;
                    q1 += t.dL1u[m] * um;
                    w0 += t.L0u[m] * wm;
                    w1v += t.L1u[m] * wm;
                    p0 += t.L0u[m] * pp[m];
                    p1 += t.L1u[m] * pp[m];
                }
                const double* recl = s_f + ((lc2 * 2) * NF + ln) * REC;
                const double* recr = s_f + ((lc2 * 2 + 1) * NF + ln) * REC;
                const bool hl = s_nbr[lc2 * 2 * DIM + 2 * a] >= 0;
                const bool hr = s_nbr[lc2 * 2 * DIM + 2 * a + 1] >= 0;
                // face averages (own trace on a boundary face)
                const double gL = hl ? 0.5 * (q0 + recl[2 * c + 1]) : q0;
                const double gR = hr ? 0.5 * (q1 + recr[2 * c + 1]) : q1;
                const double fL = hl ? 0.5 * (u0 * w0 + recl[2 * c] * recl[2 * DIM]) : u0 * w0;
                const double fR = hr ? 0.5 * (u1v * w1v + recr[2 * c] * recr[2 * DIM]) : u1v * w1v;
                const double pL = hl ? 0.5 * (p0 + recl[2 * DIM + 1]) : p0;
                const double pR = hr ? 0.5 * (p1 + recr[2 * DIM + 1]) : p1;
                double gq[N];
#pragma unroll
                for (int j = 0; j < N; ++j) {
                    double v = 0.0;
#pragma unroll
                    for (int m = 0; m < N; ++m) v += t.Du[j * N + m] * uu[m];
                    gq[j] = v;
                }
                const double wt = L::wtan(s_W, ln);
                const double kd = -cd * lg.sdiff[a] * wt, ka = ca * lg.sadv[a] * wt;
                const double kp = pl ? lg.sadv[a] * wt : 0.0;
                const double cl = kd * gL + ka * fL + kp * pL;
                const double cr = kd * gR + ka * fR + kp * pR;
#pragma unroll
                for (int i = 0; i < N; ++i) {
                    double vd = 0.0, va = 0.0, vp = 0.0;
#pragma unroll
                    for (int j = 0; j < N; ++j) {
                        const double wd = lt.WD[j * N + i];
                        vd += wd * gq[j];
                        va += wd * uw[j];
                        vp += wd * pp[j];
                    }
                    const double out = kd * vd + ka * va + kp * vp + t.L0u[i] * cl - t.L1u[i] * cr;
                    const int ni = L::node(a, i, ln);
                    s_y[c][base + ni + ni / N] += out;
                }
            }
            __syncthreads();
        }
    }
    if (active) {
#pragma unroll
        for (int c = 0; c < DIM; ++c) rhs[((size_t)cell * DIM + c) * NB + nd] = s_y[c][pi];
    }
}

// Helmholtz right-hand side (eq. helmholtz_1 and its stage-2 analogue) in
// sum-factorised form:
//   rhs_i = alpha |K| W^p_i p_prev,i
//         + f [ sum_c (|K|/h_c) sum_q W_q u_c(q) (d_c psi_i)(q)
//               - sum_faces (|K|/h_a) sum_t W_t sg {{u_a}}(t) psi_i(t) ]
// on the velocity quadrature (sg = -1 on the left face of a direction, +1 on
// the right; on a boundary face the average is the own trace).  The volume
// sum runs as one-dimensional contractions from the N^d velocity points to
// the (N-1)^d pressure nodes, one direction at a time.
template <int DIM, int N>
__global__ __launch_bounds__(256) void k_rhs_p_lines(Geom g, LineGeom lg, Tables t, double alpha,
                                                      double fcoef, const double* __restrict__ u,
                                                      const double* __restrict__ pprev,
                                                      double* __restrict__ rhs, int Nc) {
    constexpr int NP = N - 1;
    using L = Lay<DIM, N>;
    using F = FaceLay<DIM, N>;
    constexpr int NB = F::NB, NF = F::NF, CPB = F::CPB;
    constexpr int NBq = ipow(NP, DIM);
    constexpr int S1 = NP * ipow(N, DIM - 1);
    constexpr int S2 = DIM == 3 ? NP * NP * N : 1;
    constexpr int NFACE = 2 * DIM * NF;
    __shared__ double s_v[DIM][CPB * NB];
    __shared__ double s_1[DIM][CPB * S1];
    __shared__ double s_2[DIM][CPB * S2];
    __shared__ double s_face[CPB * NFACE];
    __shared__ int s_nbr[CPB * 2 * DIM];
    const int tid = threadIdx.x;
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    const int lc = tid / NB, nd = tid % NB;
    const int cell = blk * CPB + lc;
    const bool active = lc < CPB && cell < Nc;
    if (lc < CPB) {
        double wq = 1.0;
#pragma unroll
        for (int a = 0; a < DIM; ++a) wq *= t.Wu[L::coord(nd, a)];
#pragma unroll
        for (int c = 0; c < DIM; ++c)
            s_v[c][lc * NB + nd] =
                active ? wq * (g.vol / g.h[c]) * u[((size_t)cell * DIM + c) * NB + nd] : 0.0;
        if (nd == 0) {
            const Nbrs<DIM> nb(g, lg, active ? cell : 0);
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                s_nbr[lc * 2 * DIM + 2 * a] = active ? nb.left[a] : -1;
                s_nbr[lc * 2 * DIM + 2 * a + 1] = active ? nb.right[a] : -1;
            }
        }
    }
    __syncthreads();
    // face values -sg (|K|/h_a) W_t {{u_a}} at every face point of the own cells
    for (int it = tid; it < CPB * NFACE; it += 256) {
        const int lc1 = it / NFACE, face = (it / NF) % (2 * DIM), tt = it % NF;
        const int a = face >> 1, sd = face & 1;
        const int cell1 = blk * CPB + lc1;
        double val = 0.0;
        if (cell1 < Nc) {
            double uo = 0.0;
#pragma unroll
            for (int m = 0; m < N; ++m)
                uo += (sd ? t.L1u[m] : t.L0u[m]) * u[((size_t)cell1 * DIM + a) * NB + L::node(a, m, tt)];
            double uavg = uo;
            const int nbr = s_nbr[lc1 * 2 * DIM + face];
            if (nbr >= 0) {
                double un = 0.0;
#pragma unroll
                for (int m = 0; m < N; ++m)
                    un += (sd ? t.L0u[m] : t.L1u[m]) * u[((size_t)nbr * DIM + a) * NB + L::node(a, m, tt)];
                uavg = 0.5 * (uo + un);
            }
            val = -uavg * (sd ? 1.0 : -1.0) * (g.vol / g.h[a]) * L::wtan(t.Wu, tt);
        }
        s_face[it] = val;
    }
    // volume, first contraction (direction 0): [q0, q1, (q2)] -> [i0, q1, (q2)]
    for (int it = tid; it < CPB * DIM * S1; it += 256) {
        const int lc1 = it / (DIM * S1), c = (it / S1) % DIM, r = it % S1;
        const int i0 = r % NP, rest = r / NP;   // rest = q1 + N q2
        const double* B = c == 0 ? t.Dpu : t.Ip;
        double acc = 0.0;
#pragma unroll
        for (int q0 = 0; q0 < N; ++q0) acc += B[q0 * NMAX + i0] * s_v[c][lc1 * NB + q0 + N * rest];
        s_1[c][lc1 * S1 + r] = acc;
    }
    __syncthreads();
    if (DIM == 3) {
        // second contraction (direction 1): [i0, q1, q2] -> [i0, i1, q2]
        for (int it = tid; it < CPB * DIM * S2; it += 256) {
            const int lc1 = it / (DIM * S2), c = (it / S2) % DIM, r = it % S2;
            const int i0 = r % NP, i1 = (r / NP) % NP, q2 = r / (NP * NP);
            const double* B = c == 1 ? t.Dpu : t.Ip;
            double acc = 0.0;
#pragma unroll
            for (int q1 = 0; q1 < N; ++q1)
                acc += B[q1 * NMAX + i1] * s_1[c][lc1 * S1 + i0 + NP * (q1 + N * q2)];
            s_2[c][lc1 * S2 + r] = acc;
        }
        __syncthreads();
    }
    // last contraction, sum over components and the faces: one thread per
    // pressure node
    for (int it = tid; it < CPB * NBq; it += 256) {
        const int lc1 = it / NBq, i = it % NBq;
        const int cell1 = blk * CPB + lc1;
        if (cell1 >= Nc) continue;
        int ic[3] = {i % NP, (i / NP) % NP, DIM == 3 ? i / (NP * NP) : 0};
        double acc = 0.0;
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            const double* B = c == DIM - 1 ? t.Dpu : t.Ip;
#pragma unroll
            for (int q = 0; q < N; ++q) {
                const double v = DIM == 3 ? s_2[c][lc1 * S2 + ic[0] + NP * (ic[1] + NP * q)]
                                          : s_1[c][lc1 * S1 + ic[0] + NP * q];
                acc += B[q * NMAX + ic[DIM - 1]] * v;
            }
        }
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
#pragma unroll
            for (int sd = 0; sd < 2; ++sd) {
                double sum = 0.0;
                for (int tt = 0; tt < NF; ++tt) {
                    const int q = L::node(a, 0, tt);
                    double b = 1.0;
#pragma unroll
                    for (int e = 0; e < DIM; ++e)
                        if (e != a) b *= t.Ip[L::coord(q, e) * NMAX + ic[e]];
                    sum += b * s_face[lc1 * NFACE + (2 * a + sd) * NF + tt];
                }
                acc += (sd ? t.L1p[ic[a]] : t.L0p[ic[a]]) * sum;
            }
        }
        double wp = 1.0;
#pragma unroll
        for (int e = 0; e < DIM; ++e) wp *= t.Wp[ic[e]];
        const size_t gi = (size_t)cell1 * NBq + i;
        rhs[gi] = alpha * g.vol * wp * pprev[gi] + fcoef * acc;
    }
}

// Pressure operator.  MODE 0: y = H p.  MODE 3: one fused CG step: every
// block first adds the Gu partial sums (r.z, r.r) left by the previous update
// kernel (same order in every block, so all blocks agree bit for bit) and
// forms beta = rz / rz_prev (0 on the first step); the operator is then
// applied to p_new = r * invd + beta * p, evaluated on the fly for the
// neighbour traces and stored to p_out for the own cells (p_out must not
// alias p: other blocks still read the old p); one partial sum of p_new . y
// is written per block.  Block 0 records rz in sc[slot] and r.r in sc[2].
// MODE 4: the same step of flexible CG, with the preconditioned residual z
// passed in `r` and beta already in sc[5]: p_new = z + beta p.
template <int DIM, int NP, int MODE>
__global__ __launch_bounds__(256) void k_pressure_face(Geom g, LineGeom lg, Line1D lt, Tables t,
                                                        double Cr, double cm,
                                                        const double* __restrict__ p,
                                                        double* __restrict__ y, int Nc,
                                                        double* partial,
                                                        const double* __restrict__ r,
                                                        const double* __restrict__ invd,
                                                        double* __restrict__ sc,
                                                        double* __restrict__ p_out,
                                                        const double* __restrict__ up, int Gu,
                                                        int first, int slot, int slot_prev) {
    using L = Lay<DIM, NP>;
    using F = FaceLay<DIM, NP>;
    constexpr int NB = F::NB, NF = F::NF, CPB = F::CPB;
    constexpr int NFACE = 2 * DIM * NF;
    __shared__ double s_p[256];
    __shared__ double s_y[DIM][256];
    __shared__ double s_f[CPB * NFACE * 2];
    __shared__ int s_nbr[CPB * 2 * DIM];
    __shared__ double s_W[NP];
    const int tid = threadIdx.x;
    if (tid < NP) s_W[tid] = t.Wp[tid];
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    const int lc = tid / NB, nd = tid % NB;
    const int cell = blk * CPB + lc;
    const bool active = lc < CPB && cell < Nc;
    double beta = 0.0;
    if (MODE == 4) beta = sc[5];
    if (MODE == 3) {
        __shared__ double s_beta;
        double rz = 0.0, rr = 0.0;
        for (int b = tid; b < Gu; b += 256) {
            rz += up[b];
            rr += up[Gu + b];
        }
        rz = red::block_sum(rz);
        rr = red::block_sum(rr);
        if (tid == 0) {
            s_beta = first ? 0.0 : rz / sc[slot_prev];
            if (blockIdx.x == 0) {
                sc[slot] = rz;
                sc[2] = rr;
            }
        }
        __syncthreads();
        beta = s_beta;
    }
    double pown = 0.0;
    if (active) {
        const size_t gi = (size_t)cell * NB + nd;
        pown = MODE == 3 ? r[gi] * invd[gi] + beta * p[gi] : MODE == 4 ? r[gi] + beta * p[gi] : p[gi];
        if (MODE >= 3) p_out[gi] = pown;
    }
    s_p[tid] = pown;
    if (lc < CPB && nd == 0) {
        const Nbrs<DIM> nb(g, lg, active ? cell : 0);
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            s_nbr[lc * 2 * DIM + 2 * a] = active ? nb.left[a] : -1;
            s_nbr[lc * 2 * DIM + 2 * a + 1] = active ? nb.right[a] : -1;
        }
    }
    __syncthreads();
    {
        for (int it = nd; lc < CPB && it < NFACE; it += NB) {
            const int face = it / NF, tt = it % NF;
            const int a = face >> 1, s = face & 1;
            double v = 0.0, d = 0.0;
            const int nbr = s_nbr[lc * 2 * DIM + face];
            if (nbr >= 0) {
#pragma unroll
                for (int m = 0; m < NP; ++m) {
                    const size_t gi = (size_t)nbr * NB + L::node(a, m, tt);
                    const double pv = MODE == 3   ? r[gi] * invd[gi] + beta * p[gi]
                                      : MODE == 4 ? r[gi] + beta * p[gi]
                                                  : p[gi];
                    v += (s ? t.L0p[m] : t.L1p[m]) * pv;
                    d += (s ? t.dL0p[m] : t.dL1p[m]) * pv;
                }
            }
            s_f[2 * (lc * NFACE + it)] = v;
            s_f[2 * (lc * NFACE + it) + 1] = d;
        }
    }
    __syncthreads();
    constexpr int ITEMS = CPB * DIM * NF;
    for (int it = tid; it < ITEMS; it += 256) {
        const int lc2 = it / (DIM * NF);
        const int a = (it % (DIM * NF)) / NF, ln = it % NF;
        if (blk * CPB + lc2 >= Nc) continue;
        const int base = lc2 * NB;
        double pp[NP];
        double p0 = 0.0, p1 = 0.0;
#pragma unroll
        for (int m = 0; m < NP; ++m) {
            pp[m] = s_p[base + L::node(a, m, ln)];
            p0 += t.L0p[m] * pp[m];
            p1 += t.L1p[m] * pp[m];
        }
        const bool hl = s_nbr[lc2 * 2 * DIM + 2 * a] >= 0;
        const bool hr = s_nbr[lc2 * 2 * DIM + 2 * a + 1] >= 0;
        double X0, Y0, X1, Y1;
        if (hl) {
            const int rl = 2 * (lc2 * NFACE + (2 * a) * NF + ln);
            X0 = 0.5 * s_f[rl + 1] - Cr * s_f[rl];
            Y0 = 0.5 * s_f[rl];
        } else {
            // no neighbour: traces of the own cell's mirror image (LineGeom::wall)
            double q0 = 0.0;
#pragma unroll
            for (int m = 0; m < NP; ++m) q0 += t.dL0p[m] * pp[m];
            X0 = lg.wall * (0.5 * q0 + Cr * p0);
            Y0 = -lg.wall * 0.5 * p0;
        }
        if (hr) {
            const int rr = 2 * (lc2 * NFACE + (2 * a + 1) * NF + ln);
            X1 = -0.5 * s_f[rr + 1] - Cr * s_f[rr];
            Y1 = 0.5 * s_f[rr];
        } else {
            double q1 = 0.0;
#pragma unroll
            for (int m = 0; m < NP; ++m) q1 += t.dL1p[m] * pp[m];
            X1 = lg.wall * (Cr * p1 - 0.5 * q1);
            Y1 = -lg.wall * 0.5 * p1;
        }
        const double sd = lg.sdiff[a] * L::wtan(s_W, ln);
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            double s = 0.0;
#pragma unroll
            for (int j = 0; j < NP; ++j) s += lt.A[i * NP + j] * pp[j];
            s += t.L0p[i] * X0 - t.dL0p[i] * Y0 + t.L1p[i] * X1 + t.dL1p[i] * Y1;
            s_y[a][base + L::node(a, i, ln)] = sd * s;
        }
    }
    __syncthreads();
    double acc = 0.0;
    if (active) {
        acc = cm * L::wnode(s_W, nd) * pown;
#pragma unroll
        for (int a = 0; a < DIM; ++a) acc += s_y[a][tid];
        y[(size_t)cell * NB + nd] = acc;
    }
    if (MODE >= 3) {
        const double pq = red::block_sum(active ? acc * pown : 0.0);
        if (threadIdx.x == 0) partial[blockIdx.x] = pq;
    }
}

inline unsigned nblk(int64_t work, int per) { return (unsigned)((work + per - 1) / per); }

}  // namespace

#define TBDG_LINE_DISPATCH(ctx, FN)                                                       \
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

void launch_apply_pressure(const tbdg_ctx* c, double alpha, const double* p, double* y) {
    if (c->mapped) {
        map_apply_pressure(c, alpha, p, y, 0, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                           0, 0, 0, 0, nullptr);
        return;
    }
#define L_(D, N)                                                                           \
    {                                                                                      \
        using FL = FaceLay<D, N - 1>;                                                      \
        TimedLaunch tl(c, 0, 16.0 * (double)c->Np);                                        \
        hipExtLaunchKernelGGL((k_pressure_face<D, N - 1, 0>), dim3(nblk(c->Nc, FL::CPB)),  \
                              dim3(FL::THREADS), 0, c->stream, tl.start(), tl.stop(), 0,   \
                              c->geom, c->lgeom, c->line_p, c->tab, c->cr_p,               \
                              alpha * c->geom.vol, p, y, (int)c->Nc, (double*)nullptr,     \
                              (const double*)nullptr, (const double*)nullptr,              \
                              (double*)nullptr, (double*)nullptr, (const double*)nullptr,  \
                              0, 0, 0, 0);                                                 \
    }
    TBDG_LINE_DISPATCH(c, L_);
#undef L_
    TBDG_HIP(hipGetLastError());
}

void launch_diag_pressure(const tbdg_ctx* c, double alpha, double* d) {
    if (c->mapped) {
        map_diag_pressure(c, alpha, d);
        return;
    }
#define L_(D, N)                                                                           \
    hipLaunchKernelGGL((k_pressure_line<D, N - 1, 1>), dim3(nblk(c->Np, 256)), dim3(256),   \
                       0, c->stream, c->geom, c->lgeom, c->line_p, c->tab,                 \
                       alpha * c->geom.vol, nullptr, d, (int)c->Nc, nullptr);
    TBDG_LINE_DISPATCH(c, L_);
#undef L_
    TBDG_HIP(hipGetLastError());
}

int launch_cg_apply(const tbdg_ctx* c, double alpha, const double* r, const double* invd,
                    const double* p_old, double* p_new, double* q, double* sc, const double* up,
                    int Gu, int first, int slot, int slot_prev) {
    int G = 0;
    if (c->mapped) {
        map_apply_pressure(c, alpha, p_old, q, 3, c->red_op, r, invd, sc, p_new, up, Gu, first,
                           slot, slot_prev, &G);
        return G;
    }
#define L_(D, N)                                                                           \
    {                                                                                      \
        using FL = FaceLay<D, N - 1>;                                                      \
        G = (int)nblk(c->Nc, FL::CPB);                                                     \
        if (G > c->red_op_len) throw Error(TBDG_EINVAL, "operator partial buffer too small"); \
        TimedLaunch tl(c, 0, 40.0 * (double)c->Np);                                        \
        hipExtLaunchKernelGGL((k_pressure_face<D, N - 1, 3>), dim3(G), dim3(FL::THREADS),  \
                              0, c->stream, tl.start(), tl.stop(), 0, c->geom, c->lgeom,   \
                              c->line_p, c->tab, c->cr_p, alpha * c->geom.vol, p_old, q,  \
                              (int)c->Nc, c->red_op, r, invd, sc, p_new, up, Gu, first,    \
                              slot, slot_prev);                                            \
    }
    TBDG_LINE_DISPATCH(c, L_);
#undef L_
    TBDG_HIP(hipGetLastError());
    return G;
}

// Pressure-type operator of one multigrid level (FP64): any node count np
// per direction (2..5 in 2D, 2..3 in 3D) with the level's own geometry.
#define TBDG_NP_DISPATCH(dim, np, FN)                                                    \
    do {                                                                                  \
        if ((dim) == 2 && (np) == 2) { FN(2, 2); }                                        \
        else if ((dim) == 2 && (np) == 3) { FN(2, 3); }                                   \
        else if ((dim) == 2 && (np) == 4) { FN(2, 4); }                                   \
        else if ((dim) == 2 && (np) == 5) { FN(2, 5); }                                   \
        else if ((dim) == 2 && (np) == 6) { FN(2, 6); }                                   \
        else if ((dim) == 3 && (np) == 2) { FN(3, 2); }                                   \
        else if ((dim) == 3 && (np) == 3) { FN(3, 3); }                                   \
        else if ((dim) == 3 && (np) == 4) { FN(3, 4); }                                   \
        else throw Error(TBDG_EUNSUPPORTED, "unsupported (dim, pressure nodes)");          \
    } while (0)

void launch_pressure_level(hipStream_t s, int dim, int np, const Geom& g, const LineGeom& lg,
                           const Line1D& lt, const Tables& t, double cr, double cm,
                           const double* p, double* y, int64_t Nc) {
#define L_(D, NP)                                                                          \
    {                                                                                      \
        using FL = FaceLay<D, NP>;                                                         \
        hipLaunchKernelGGL((k_pressure_face<D, NP, 0>), dim3(nblk(Nc, FL::CPB)),           \
                           dim3(FL::THREADS), 0, s, g, lg, lt, t, cr, cm, p, y, (int)Nc,   \
                           (double*)nullptr, (const double*)nullptr, (const double*)nullptr, \
                           (double*)nullptr, (double*)nullptr, (const double*)nullptr, 0, \
                           0, 0, 0);                                                       \
    }
    TBDG_NP_DISPATCH(dim, np, L_);
#undef L_
    TBDG_HIP(hipGetLastError());
}

void launch_diag_pressure_level(hipStream_t s, int dim, int np, const Geom& g, const LineGeom& lg,
                                const Line1D& lt, const Tables& t, double cm, double* d,
                                int64_t Nc) {
#define L_(D, NP)                                                                          \
    hipLaunchKernelGGL((k_pressure_line<D, NP, 1>), dim3(nblk(Nc * ipow(NP, D), 256)),     \
                       dim3(256), 0, s, g, lg, lt, t, cm, nullptr, d, (int)Nc, nullptr);
    TBDG_NP_DISPATCH(dim, np, L_);
#undef L_
    TBDG_HIP(hipGetLastError());
}

int launch_fcg_apply(const tbdg_ctx* c, double alpha, const double* z, const double* p_old,
                     double* p_new, double* q, double* sc) {
    int G = 0;
    if (c->mapped) {
        map_apply_pressure(c, alpha, p_old, q, 4, c->red_op, z, nullptr, sc, p_new, nullptr, 0, 0,
                           0, 0, &G);
        return G;
    }
#define L_(D, N)                                                                           \
    {                                                                                      \
        using FL = FaceLay<D, N - 1>;                                                      \
        G = (int)nblk(c->Nc, FL::CPB);                                                     \
        if (G > c->red_op_len) throw Error(TBDG_EINVAL, "operator partial buffer too small"); \
        TimedLaunch tl(c, 0, 32.0 * (double)c->Np);                                        \
        hipExtLaunchKernelGGL((k_pressure_face<D, N - 1, 4>), dim3(G), dim3(FL::THREADS),  \
                              0, c->stream, tl.start(), tl.stop(), 0, c->geom, c->lgeom,   \
                              c->line_p, c->tab, c->cr_p, alpha * c->geom.vol, p_old, q,  \
                              (int)c->Nc, c->red_op, z, (const double*)nullptr, sc, p_new, \
                              (const double*)nullptr, 0, 0, 0, 0);                         \
    }
    TBDG_LINE_DISPATCH(c, L_);
#undef L_
    TBDG_HIP(hipGetLastError());
    return G;
}

int launch_apply_momentum_fused(const tbdg_ctx* c, int st, const double* w, const double* u,
                                double* y, const MomFuse& fz) {
    const double mcoef = c->mcoef(st), theta = c->theta[st];
    const Bnd bd = c->bnd(st);
    if (fz.ndot < 0 || fz.ndot > MOM_FUSE_MAX_DOTS)
        throw Error(TBDG_EINVAL, "fused dot count out of range");
    if (c->mapped) return map_apply_momentum(c, st, w, u, y, fz);
    int G = 0;
    // algorithmic bytes: read u and w, write y; fused: the inverse diagonal
    // and the basis vectors of the dots
    double bytes = 24.0 * (double)c->Nu;
    if (fz.invd) bytes += 8.0 * (double)c->Ns;
    if (fz.shv) bytes += 8.0 * (double)c->Nu;
    bytes += 8.0 * fz.ndot * (double)c->Nu;
    if (fz.rb) bytes += 8.0 * (double)c->Nu;
#define L_(D, N)                                                                           \
    {                                                                                      \
        using FL = FaceLay<D, N>;                                                          \
        G = (int)nblk(c->Nc, FL::CPB);                                                     \
        if (fz.ndot > 0 && (int64_t)G * (fz.ndot + 1) > c->gm_part_len)                    \
            throw Error(TBDG_EINVAL, "fused partial buffer too small");                    \
        TimedLaunch tl(c, 1, bytes);                                                       \
        hipExtLaunchKernelGGL((k_momentum_face<D, N>), dim3(G), dim3(FL::THREADS), 0,      \
                              c->stream, tl.start(), tl.stop(), 0, c->geom, c->lgeom,      \
                              c->line_u, c->tab, c->cr_u, mcoef * c->geom.vol,             \
                              theta * c->nu, theta, w, u, y, (int)c->Nc, bd, fz,           \
                              tile_zchunk(c->dim, c->geom.nc, FL::CPB));                   \
    }
    TBDG_LINE_DISPATCH(c, L_);
#undef L_
    TBDG_HIP(hipGetLastError());
    return G;
}

void launch_apply_momentum(const tbdg_ctx* c, int st, const double* w, const double* u, double* y) {
    launch_apply_momentum_fused(c, st, w, u, y,
                                MomFuse{nullptr, nullptr, 0.0, nullptr, 0, 0, nullptr, nullptr});
}

void launch_residual_momentum(const tbdg_ctx* c, int st, const double* w, const double* u,
                              const double* b, double* r) {
    if (c->mapped) {
        // the mapped kernels have no residual mode: apply, then subtract
        launch_apply_momentum(c, st, w, u, r);
        vec_axpby(c->stream, c->Nu, 1.0, b, -1.0, r, r);
        return;
    }
    MomFuse fz{nullptr, nullptr, 0.0, nullptr, 0, 0, nullptr, nullptr};
    fz.rb = b;
    launch_apply_momentum_fused(c, st, w, u, r, fz);
}

void launch_rhs_lines(const tbdg_ctx* c, double mcoef, const double* u_prev, const double* u1,
                      const double* w1, double cd1, double ca1, const double* u2, const double* w2,
                      double cd2, double ca2, const double* pv, double* rhs) {
#define L_(D, N)                                                                           \
    {                                                                                      \
        using FL = FaceLay<D, N>;                                                          \
        hipLaunchKernelGGL((k_rhs_lines<D, N>), dim3(nblk(c->Nc, FL::CPB)), dim3(FL::THREADS), \
                           0, c->stream, c->geom, c->lgeom, c->line_u, c->tab,             \
                           mcoef * c->geom.vol, u_prev, u1, w1, cd1, ca1, u2, w2, cd2, ca2, \
                           pv, rhs, (int)c->Nc);                                           \
    }
    TBDG_LINE_DISPATCH(c, L_);
#undef L_
    TBDG_HIP(hipGetLastError());
}

void launch_rhs_p_lines(const tbdg_ctx* c, double alpha, double fcoef, const double* u_ss,
                        const double* p_prev, double* rhs) {
#define L_(D, N)                                                                           \
    {                                                                                      \
        using FL = FaceLay<D, N>;                                                          \
        hipLaunchKernelGGL((k_rhs_p_lines<D, N>), dim3(nblk(c->Nc, FL::CPB)), dim3(FL::THREADS), \
                           0, c->stream, c->geom, c->lgeom, c->tab, alpha, fcoef, u_ss, p_prev, \
                           rhs, (int)c->Nc);                                               \
    }
    TBDG_LINE_DISPATCH(c, L_);
#undef L_
    TBDG_HIP(hipGetLastError());
}

// On Q1-mapped cells the blocks are those of the undistorted box (c->geom),
// built with that box's diagonal (launch_diag_momentum_box): a fixed
// approximation of the distorted operator, spectrally close to it while the
// map is a small perturbation of the identity.
void launch_mom_lineblk(const tbdg_ctx* c, int st, const double* w, const double* d,
                        float* blk) {
    const double theta = c->theta[st];
    const Bnd bd = c->bnd(st);
#define L_(D, N)                                                                           \
    {                                                                                      \
        const int64_t items = c->Nc * D * ipow(N, D - 1);                                  \
        hipLaunchKernelGGL((k_mom_lineblk<D, N>), dim3((unsigned)((items + 255) / 256)),    \
                           dim3(256), 0, c->stream, c->geom, c->lgeom, c->line_u, c->tab,   \
                           c->cr_u, theta * c->nu, theta, w, d, blk, (int)c->Nc, bd);       \
    }
    TBDG_LINE_DISPATCH(c, L_);
#undef L_
    TBDG_HIP(hipGetLastError());
}

void launch_mom_lineprec(const tbdg_ctx* c, const float* blk, const double* d, const double* v,
                         const double* scale, double* z, bool accumulate) {
#define L_(D, N)                                                                           \
    {                                                                                      \
        using FL = FaceLay<D, N>;                                                          \
        hipLaunchKernelGGL((k_mom_lineprec<D, N>), dim3(nblk(c->Nc, FL::CPB)),              \
                           dim3(FL::THREADS), 0, c->stream, blk, d, v, scale, z, (int)c->Nc, \
                           accumulate ? 1 : 0);                                            \
    }
    TBDG_LINE_DISPATCH(c, L_);
#undef L_
    TBDG_HIP(hipGetLastError());
}

void launch_diag_momentum(const tbdg_ctx* c, int st, const double* w, double* d) {
    if (c->mapped) {
        map_diag_momentum(c, st, w, d);
        return;
    }
    launch_diag_momentum_box(c, st, w, d);
}

void launch_diag_momentum_box(const tbdg_ctx* c, int st, const double* w, double* d) {
    const double mcoef = c->mcoef(st), theta = c->theta[st];
    const Bnd bd = c->bnd(st);
#define L_(D, N)                                                                           \
    {                                                                                      \
        using LL = Lay<D, N>;                                                              \
        hipLaunchKernelGGL((k_momentum_line<D, N, true>), dim3(nblk(c->Nc, LL::CPB)),      \
                           dim3(LL::THREADS), 0, c->stream, c->geom, c->lgeom, c->line_u,  \
                           c->tab, mcoef * c->geom.vol, theta * c->nu, theta, w, nullptr,  \
                           d, (int)c->Nc, bd);                                             \
    }
    TBDG_LINE_DISPATCH(c, L_);
#undef L_
    TBDG_HIP(hipGetLastError());
}

}  // namespace trbdg
