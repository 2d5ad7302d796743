// Matrix-free DG operators on Q1-mapped quadrilaterals (2D) for gfx950.
//
// Each cell is the bilinear image of the reference square through its four
// vertices (Sec. 3: hexahedral / quadrilateral cells mapped from the
// reference cell).  The Jacobian J(xi) is recomputed in the kernels from the
// vertices; with adj(J) = det(J) J^{-1}:
//   physical gradient      grad u = adj(J)^T grad_xi u / det J,
//   diffusion flux         W det grad u . grad v = grad_xi v . (W / det) adj adj^T grad_xi u,
//   advection flux         W det u (w . grad v)  = grad_xi v . (W u adj w),
//   face normal / weight   n = +-row_a(adj) / |row_a(adj)|, dS = W_t |row_a(adj)|
// (Nanson's formula; the edges of a Q1 quadrilateral are straight, so n and
// dS are constant along a face).  The Lagrange bases sit at the Gauss points
// of the quadrature rule (collocation), so the volume terms are contractions
// of per-point contravariant fluxes with the 1D derivative matrix.
//
// Layout as on the affine box: velocity [cell][component][node], pressure
// [cell][node], cells lexicographic (x fastest).  A work-group owns CPB whole
// cells, one thread per node; the face terms of all four faces are evaluated
// by each cell for its own side, with the neighbour's trace and normal
// derivative recomputed from the neighbour's values in global memory, so
// every output is written by exactly one thread (no atomics, bitwise
// reproducible).
#include "internal.hpp"
#include "reduce.hpp"

#include <hip/hip_ext.h>

namespace trbdg {
namespace {

constexpr int mcpb(int nb) { return (256 / nb) < 16 ? (256 / nb) : 16; }

// node index of coordinate m along direction a, tangential index t
template <int N>
__device__ inline int mnode(int a, int m, int t) {
    return a == 0 ? m + N * t : t + N * m;
}

// adj(J) = [[m00, m01], [m10, m11]] and det J of the bilinear map of the
// vertices X (vertex v = vx + 2 vy at X[2v], X[2v+1]) at (x0, x1)
struct Adj {
    double m00, m01, m10, m11, det;
};

__device__ inline Adj map_adj(const double* X, double x0, double x1) {
    const double j00 = (1.0 - x1) * (X[2] - X[0]) + x1 * (X[6] - X[4]);   // dx/dxi0
    const double j10 = (1.0 - x1) * (X[3] - X[1]) + x1 * (X[7] - X[5]);   // dy/dxi0
    const double j01 = (1.0 - x0) * (X[4] - X[0]) + x0 * (X[6] - X[2]);   // dx/dxi1
    const double j11 = (1.0 - x0) * (X[5] - X[1]) + x0 * (X[7] - X[3]);   // dy/dxi1
    return Adj{j11, -j01, -j10, j00, j00 * j11 - j01 * j10};
}

// Face (a, s) of a cell at tangential reference coordinate xt with weight wt:
// outward unit normal, surface weight, and the reference-gradient weights
// (va along a, vb along the tangential direction) of the normal derivative,
// grad u . n = va d_a u + vb d_b u (J^{-1} n).
struct FaceG {
    double n0, n1, dS, va, vb;
};

__device__ inline FaceG face_geo(const double* X, int a, int s, double xt, double wt) {
    const double x0 = a == 0 ? (double)s : xt, x1 = a == 0 ? xt : (double)s;
    const Adj J = map_adj(X, x0, x1);
    const double r0 = a == 0 ? J.m00 : J.m10, r1 = a == 0 ? J.m01 : J.m11;
    const double len = sqrt(r0 * r0 + r1 * r1);
    const double sg = s ? 1.0 : -1.0;
    FaceG f;
    f.n0 = sg * r0 / len;
    f.n1 = sg * r1 / len;
    f.dS = wt * len;
    const double v0 = (J.m00 * f.n0 + J.m01 * f.n1) / J.det;
    const double v1 = (J.m10 * f.n0 + J.m11 * f.n1) / J.det;
    f.va = a == 0 ? v0 : v1;
    f.vb = a == 0 ? v1 : v0;
    return f;
}

// The neighbour's reference-gradient weights of its own outward normal -n at
// its face (a, 1 - s), point xt.
__device__ inline void nbr_ref(const double* XN, int a, int s, double xt, double n0, double n1,
                               double& va, double& vb) {
    const double xs = (double)(1 - s);
    const double x0 = a == 0 ? xs : xt, x1 = a == 0 ? xt : xs;
    const Adj J = map_adj(XN, x0, x1);
    const double v0 = -(J.m00 * n0 + J.m01 * n1) / J.det;
    const double v1 = -(J.m10 * n0 + J.m11 * n1) / J.det;
    va = a == 0 ? v0 : v1;
    vb = a == 0 ? v1 : v0;
}

__device__ inline int map_nbr(const MapMesh& m, int cell, int f) {
    const int a = f >> 1, s = f & 1;
    int c0 = cell % m.nc[0], c1 = cell / m.nc[0];
    if (a == 0) {
        c0 += s ? 1 : -1;
        if (c0 < 0 || c0 >= m.nc[0]) {
            if (!m.per[0]) return -1;
            c0 = (c0 + m.nc[0]) % m.nc[0];
        }
    } else {
        c1 += s ? 1 : -1;
        if (c1 < 0 || c1 >= m.nc[1]) {
            if (!m.per[1]) return -1;
            c1 = (c1 + m.nc[1]) % m.nc[1];
        }
    }
    return c0 + m.nc[0] * c1;
}

// boundary point index of face point t on face (a, s) of `cell`
__device__ inline int64_t map_bnd_point(const MapMesh& m, int cell, int a, int s, int t, int N) {
    const int tc = a == 0 ? cell / m.nc[0] : cell % m.nc[0];
    return m.off[a][s] + (int64_t)tc * N + t;
}

// Stages the vertices of the block's cells, their face neighbours and the
// neighbours' vertices in LDS.  Ends with a barrier.
template <int CPB>
__device__ inline void stage_geometry(const MapMesh& mm, int cell0, int Nc, double* s_X,
                                      double* s_XN, int* s_nb) {
    const int tid = threadIdx.x;
    for (int it = tid; it < CPB * 8; it += blockDim.x) {
        const int c = cell0 + it / 8;
        s_X[it] = c < Nc ? mm.vtx[(size_t)c * 8 + it % 8] : 0.0;
    }
    for (int it = tid; it < CPB * 4; it += blockDim.x) {
        const int c = cell0 + it / 4;
        s_nb[it] = c < Nc ? map_nbr(mm, c, it % 4) : -1;
    }
    __syncthreads();
    if (s_XN) {
        for (int it = tid; it < CPB * 32; it += blockDim.x) {
            const int nb = s_nb[it / 8];
            s_XN[it] = nb >= 0 ? mm.vtx[(size_t)nb * 8 + it % 8] : 0.0;
        }
        __syncthreads();
    }
}

// ============================================================================
// Pressure operator H = alpha M^p + K (the SIP form a_p, interior faces only:
// homogeneous Neumann on boundary faces).  MODE 0: y = H p.  MODE 3: one
// fused CG step (beta from the Gu partial sums of the previous update kernel,
// p_new = r invd + beta p evaluated on the fly, stored to p_out for the own
// cells, per-block partial of p_new . y).  MODE 4: flexible CG, p_new =
// z + sc[5] p with z passed in r.
// ============================================================================
template <int NP, int MODE>
__global__ __launch_bounds__(256) void k_map_pres(MapMesh mm, Tables t, double fac, double alpha,
                                                   const double* __restrict__ p,
                                                   double* __restrict__ y, int Nc,
                                                   double* partial, const double* __restrict__ r,
                                                   const double* __restrict__ invd,
                                                   double* __restrict__ sc,
                                                   double* __restrict__ p_out,
                                                   const double* __restrict__ up, int Gu, int first,
                                                   int slot, int slot_prev) {
    constexpr int NB = NP * NP, CPB = mcpb(NB), NFP = 4 * NP, NREC = CPB * NFP;
    static_assert(NREC <= 256, "one face point per thread");
    __shared__ double s_X[CPB * 8];
    __shared__ double s_XN[CPB * 32];
    __shared__ int s_nb[CPB * 4];
    __shared__ double s_u[256];
    __shared__ double s_F[2][256];
    __shared__ double s_A[4][256];
    __shared__ double s_B[3][256];
    const int tid = threadIdx.x;
    const int lc = tid / NB, nd = tid % NB;
    const int cell0 = blockIdx.x * CPB;
    const int cell = cell0 + lc;
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
    auto opnd = [&](size_t gi) -> double {
        return MODE == 3 ? r[gi] * invd[gi] + beta * p[gi] : MODE == 4 ? r[gi] + beta * p[gi] : p[gi];
    };
    double pown = 0.0;
    if (active) {
        const size_t gi = (size_t)cell * NB + nd;
        pown = opnd(gi);
        if (MODE >= 3) p_out[gi] = pown;
    }
    s_u[tid] = pown;
    stage_geometry<CPB>(mm, cell0, Nc, s_X, s_XN, s_nb);
    const double* D = t.Dp;
    double mass = 0.0;
    if (active) {
        const int q0 = nd % NP, q1 = nd / NP, base = lc * NB;
        double g0 = 0.0, g1 = 0.0;
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            g0 += D[q0 * NP + j] * s_u[base + j + NP * q1];
            g1 += D[q1 * NP + j] * s_u[base + q0 + NP * j];
        }
        const Adj J = map_adj(s_X + lc * 8, t.xp[q0], t.xp[q1]);
        const double W = t.Wp[q0] * t.Wp[q1], wd = W / J.det;
        const double P00 = J.m00 * J.m00 + J.m01 * J.m01, P01 = J.m00 * J.m10 + J.m01 * J.m11,
                     P11 = J.m10 * J.m10 + J.m11 * J.m11;
        s_F[0][tid] = wd * (P00 * g0 + P01 * g1);
        s_F[1][tid] = wd * (P01 * g0 + P11 * g1);
        mass = alpha * W * J.det * pown;
    }
    // face records: own and neighbour trace and derivative along a
    const int lf = tid / NFP, f = (tid % NFP) / NP, tt = tid % NP;
    const int a = f >> 1, s = f & 1;
    const bool frec = tid < NREC && cell0 + lf < Nc;
    if (frec) {
        const double* Ls = s ? t.L1p : t.L0p;
        const double* dLs = s ? t.dL1p : t.dL0p;
        double uK = 0.0, dK = 0.0, uN = 0.0, dN = 0.0;
#pragma unroll
        for (int m = 0; m < NP; ++m) {
            const double v = s_u[lf * NB + mnode<NP>(a, m, tt)];
            uK += Ls[m] * v;
            dK += dLs[m] * v;
        }
        const int nb = s_nb[lf * 4 + f];
        if (nb >= 0) {
            const double* Ln = s ? t.L0p : t.L1p;
            const double* dLn = s ? t.dL0p : t.dL1p;
#pragma unroll
            for (int m = 0; m < NP; ++m) {
                const double v = opnd((size_t)nb * NB + mnode<NP>(a, m, tt));
                uN += Ln[m] * v;
                dN += dLn[m] * v;
            }
        }
        s_A[0][tid] = uK;
        s_A[1][tid] = dK;
        s_A[2][tid] = uN;
        s_A[3][tid] = dN;
    }
    __syncthreads();
    if (frec) {
        const int rb = lf * NFP + f * NP;
        double tK = 0.0, tN = 0.0;
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            tK += D[tt * NP + j] * s_A[0][rb + j];
            tN += D[tt * NP + j] * s_A[2][rb + j];
        }
        const int nb = s_nb[lf * 4 + f];
        double V = 0.0, Ga = 0.0, Gb = 0.0;
        if (nb >= 0) {
            const FaceG G = face_geo(s_X + lf * 8, a, s, t.xp[tt], t.Wp[tt]);
            double va2, vb2;
            nbr_ref(s_XN + (lf * 4 + f) * 8, a, s, t.xp[tt], G.n0, G.n1, va2, vb2);
            const double ndK = G.va * s_A[1][tid] + G.vb * tK;
            const double ndN = va2 * s_A[3][tid] + vb2 * tN;
            const double C = 0.5 * fac * (mm.gr[(size_t)(cell0 + lf) * 4 + f] + mm.gr[(size_t)nb * 4 + (f ^ 1)]);
            const double jump = s_A[0][tid] - s_A[2][tid];
            V = G.dS * (-0.5 * (ndK - ndN) + C * jump);
            Ga = 0.5 * G.dS * jump * G.va;
            Gb = 0.5 * G.dS * jump * G.vb;
        }
        s_B[0][tid] = V;
        s_B[1][tid] = Ga;
        s_B[2][tid] = Gb;
    }
    __syncthreads();
    double acc = 0.0;
    if (active) {
        const int i0 = nd % NP, i1 = nd / NP, base = lc * NB;
        acc = mass;
#pragma unroll
        for (int q = 0; q < NP; ++q)
            acc += D[q * NP + i0] * s_F[0][base + q + NP * i1] + D[q * NP + i1] * s_F[1][base + i0 + NP * q];
#pragma unroll
        for (int ff = 0; ff < 4; ++ff) {
            const int aa = ff >> 1, ss = ff & 1;
            const int ia = aa == 0 ? i0 : i1, ib = aa == 0 ? i1 : i0;
            const double L = (ss ? t.L1p : t.L0p)[ia], dL = (ss ? t.dL1p : t.dL0p)[ia];
            const int rb = lc * NFP + ff * NP;
            double g = 0.0;
#pragma unroll
            for (int q = 0; q < NP; ++q) g += D[q * NP + ib] * s_B[2][rb + q];
            acc += L * (s_B[0][rb + ib] - g) - dL * s_B[1][rb + ib];
        }
        y[(size_t)cell * NB + nd] = acc;
    }
    if (MODE >= 3) {
        const double pq = red::block_sum(active ? acc * pown : 0.0);
        if (tid == 0) partial[blockIdx.x] = pq;
    }
}

// ============================================================================
// Momentum operator of stage s, y = m M u + theta (nu A_SIP u + C_LF(w) u),
// all components in one pass (eq. bilin_diff with boundary penalty 2C,
// eq. trilinear with lambda = max(|w+.n|, |w-.n|) per face point and the
// mirrored exterior advector 2 u_D - w on Dirichlet faces), with the fused
// GMRES work of MomFuse (operand scaling, shift, partial dots).
// ============================================================================
template <int N>
__global__ __launch_bounds__(256) void k_map_mom(MapMesh mm, Tables t, double fac, double mc,
                                                  double tnu, double th,
                                                  const double* __restrict__ w,
                                                  const double* __restrict__ u,
                                                  double* __restrict__ y, int Nc, MomFuse fz) {
    constexpr int NB = N * N, CPB = mcpb(NB), NFP = 4 * N, NREC = CPB * NFP;
    static_assert(NREC <= 256, "one face point per thread");
    __shared__ double s_X[CPB * 8];
    __shared__ double s_XN[CPB * 32];
    __shared__ int s_nb[CPB * 4];
    __shared__ double s_u[2][256];
    __shared__ double s_w[2][256];
    __shared__ double s_F[2][2][256];
    __shared__ double s_A[12][256];   // uK[2] dK[2] uN[2] dN[2] wK[2] wN[2]
    // face fluxes V[2] Ga[2] Gb[2], written between the two barriers: V and
    // Ga over wK, wN (each thread reads only its own entries of those, and
    // before it writes), Gb over s_u (last read before the first barrier).
    // Keeps the block under 53 KB of LDS: three blocks per CU.
    double* const s_B[6] = {s_A[8], s_A[9], s_A[10], s_A[11], s_u[0], s_u[1]};
    const int tid = threadIdx.x;
    const int lc = tid / NB, nd = tid % NB;
    const int cell0 = blockIdx.x * CPB;
    const int cell = cell0 + lc;
    const bool active = lc < CPB && cell < Nc;
    const double us = fz.invd ? fz.gsc[0] : 1.0;
    auto scale = [&](size_t node) -> double { return fz.invd ? us * fz.invd[node] : 1.0; };
    double uraw[2] = {0.0, 0.0};
    {
        const double sc = active ? scale((size_t)cell * NB + nd) : 0.0;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const size_t gi = ((size_t)cell * 2 + c) * NB + nd;
            uraw[c] = active ? u[gi] : 0.0;
            s_u[c][tid] = uraw[c] * sc;
            s_w[c][tid] = active ? w[gi] : 0.0;
        }
    }
    stage_geometry<CPB>(mm, cell0, Nc, s_X, s_XN, s_nb);
    const double* D = t.Du;
    double mass[2] = {0.0, 0.0};
    if (active) {
        const int q0 = nd % N, q1 = nd / N, base = lc * NB;
        const Adj J = map_adj(s_X + lc * 8, t.xu[q0], t.xu[q1]);
        const double W = t.Wu[q0] * t.Wu[q1], wd = W / J.det;
        const double P00 = J.m00 * J.m00 + J.m01 * J.m01, P01 = J.m00 * J.m10 + J.m01 * J.m11,
                     P11 = J.m10 * J.m10 + J.m11 * J.m11;
        const double w0 = s_w[0][tid], w1 = s_w[1][tid];
        const double c0 = W * (J.m00 * w0 + J.m01 * w1), c1 = W * (J.m10 * w0 + J.m11 * w1);
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            double g0 = 0.0, g1 = 0.0;
#pragma unroll
            for (int j = 0; j < N; ++j) {
                g0 += D[q0 * N + j] * s_u[c][base + j + N * q1];
                g1 += D[q1 * N + j] * s_u[c][base + q0 + N * j];
            }
            const double uq = s_u[c][tid];
            s_F[c][0][tid] = tnu * wd * (P00 * g0 + P01 * g1) - th * uq * c0;
            s_F[c][1][tid] = tnu * wd * (P01 * g0 + P11 * g1) - th * uq * c1;
            mass[c] = mc * W * J.det * uq;
        }
    }
    const int lf = tid / NFP, f = (tid % NFP) / N, tt = tid % N;
    const int a = f >> 1, s = f & 1;
    const int fcell = cell0 + lf;
    const bool frec = tid < NREC && fcell < Nc;
    if (frec) {
        const double* Ls = s ? t.L1u : t.L0u;
        const double* dLs = s ? t.dL1u : t.dL0u;
        const int nb = s_nb[lf * 4 + f];
        const double* Ln = s ? t.L0u : t.L1u;
        const double* dLn = s ? t.dL0u : t.dL1u;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            double uK = 0.0, dK = 0.0, wK = 0.0, uN = 0.0, dN = 0.0, wN = 0.0;
#pragma unroll
            for (int m = 0; m < N; ++m) {
                const int li = lf * NB + mnode<N>(a, m, tt);
                uK += Ls[m] * s_u[c][li];
                dK += dLs[m] * s_u[c][li];
                wK += Ls[m] * s_w[c][li];
            }
            if (nb >= 0) {
#pragma unroll
                for (int m = 0; m < N; ++m) {
                    const int ln = mnode<N>(a, m, tt);
                    const size_t gi = ((size_t)nb * 2 + c) * NB + ln;
                    const double v = u[gi] * scale((size_t)nb * NB + ln);
                    uN += Ln[m] * v;
                    dN += dLn[m] * v;
                    wN += Ln[m] * w[gi];
                }
            }
            s_A[0 + c][tid] = uK;
            s_A[2 + c][tid] = dK;
            s_A[4 + c][tid] = uN;
            s_A[6 + c][tid] = dN;
            s_A[8 + c][tid] = wK;
            s_A[10 + c][tid] = wN;
        }
    }
    __syncthreads();
    if (frec) {
        const int rb = lf * NFP + f * N;
        const int nb = s_nb[lf * 4 + f];
        const FaceG G = face_geo(s_X + lf * 8, a, s, t.xu[tt], t.Wu[tt]);
        const double wnK = s_A[8][tid] * G.n0 + s_A[9][tid] * G.n1;
        if (nb >= 0) {
            double va2, vb2;
            nbr_ref(s_XN + (lf * 4 + f) * 8, a, s, t.xu[tt], G.n0, G.n1, va2, vb2);
            const double wnN = s_A[10][tid] * G.n0 + s_A[11][tid] * G.n1;
            const double lam = fmax(fabs(wnK), fabs(wnN));
            const double C = 0.5 * fac * (mm.gr[(size_t)fcell * 4 + f] + mm.gr[(size_t)nb * 4 + (f ^ 1)]);
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                double tK = 0.0, tN = 0.0;
#pragma unroll
                for (int j = 0; j < N; ++j) {
                    tK += D[tt * N + j] * s_A[0 + c][rb + j];
                    tN += D[tt * N + j] * s_A[4 + c][rb + j];
                }
                const double uK = s_A[0 + c][tid], uN = s_A[4 + c][tid];
                const double ndK = G.va * s_A[2 + c][tid] + G.vb * tK;
                const double ndN = va2 * s_A[6 + c][tid] + vb2 * tN;
                const double jump = uK - uN;
                s_B[0 + c][tid] = G.dS * (tnu * (-0.5 * (ndK - ndN) + C * jump) +
                                          th * (0.5 * (wnK * uK + wnN * uN) + 0.5 * lam * jump));
                s_B[2 + c][tid] = 0.5 * tnu * G.dS * jump * G.va;
                s_B[4 + c][tid] = 0.5 * tnu * G.dS * jump * G.vb;
            }
        } else {
            const int64_t pt = map_bnd_point(mm, fcell, a, s, tt, N);
            const double e0 = 2.0 * mm.uD[pt * 2] - s_A[8][tid];
            const double e1 = 2.0 * mm.uD[pt * 2 + 1] - s_A[9][tid];
            const double lam = fmax(fabs(wnK), fabs(e0 * G.n0 + e1 * G.n1));
            const double C = fac * mm.gr[(size_t)fcell * 4 + f];
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                double tK = 0.0;
#pragma unroll
                for (int j = 0; j < N; ++j) tK += D[tt * N + j] * s_A[0 + c][rb + j];
                const double uK = s_A[0 + c][tid];
                const double ndK = G.va * s_A[2 + c][tid] + G.vb * tK;
                s_B[0 + c][tid] = G.dS * (tnu * (-ndK + 2.0 * C * uK) + th * lam * uK);
                s_B[2 + c][tid] = tnu * G.dS * uK * G.va;
                s_B[4 + c][tid] = tnu * G.dS * uK * G.vb;
            }
        }
    }
    __syncthreads();
    double yv[2] = {0.0, 0.0};
    if (active) {
        const int i0 = nd % N, i1 = nd / N, base = lc * NB;
        if (fz.shv) {
#pragma unroll
            for (int c = 0; c < 2; ++c) uraw[c] = fz.shv[((size_t)cell * 2 + c) * NB + nd];
        }
        const double ysh = fz.invd ? fz.shift * us : (fz.shv ? fz.shift * fz.gsc[0] : 0.0);
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            double acc = mass[c];
#pragma unroll
            for (int q = 0; q < N; ++q)
                acc += D[q * N + i0] * s_F[c][0][base + q + N * i1] +
                       D[q * N + i1] * s_F[c][1][base + i0 + N * q];
#pragma unroll
            for (int ff = 0; ff < 4; ++ff) {
                const int aa = ff >> 1, ss = ff & 1;
                const int ia = aa == 0 ? i0 : i1, ib = aa == 0 ? i1 : i0;
                const double L = (ss ? t.L1u : t.L0u)[ia], dL = (ss ? t.dL1u : t.dL0u)[ia];
                const int rb = lc * NFP + ff * N;
                double g = 0.0;
#pragma unroll
                for (int q = 0; q < N; ++q) g += D[q * N + ib] * s_B[4 + c][rb + q];
                acc += L * (s_B[0 + c][rb + ib] - g) - dL * s_B[2 + c][rb + ib];
            }
            yv[c] = acc - ysh * uraw[c];
            y[((size_t)cell * 2 + c) * NB + nd] = yv[c];
        }
    }
    if (fz.ndot > 0) {
        __shared__ double s_red[MOM_FUSE_MAX_DOTS + 1][4];
        const int lane = tid & 63, wv = tid >> 6;
        for (int i = 0; i <= fz.ndot; ++i) {
            double v = 0.0;
            if (active) {
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    const size_t gi = ((size_t)cell * 2 + c) * NB + nd;
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

// ============================================================================
// Exact diagonals.  Pressure (MOM false): alpha M^p + K.  Momentum (MOM true):
// m M + theta (nu A_SIP + C_LF(w)), one value per scalar node (the operator
// is the identity over components times one scalar operator).  One thread
// per node; the volume part sums the squared derivative-matrix entries with
// the metric, the face part the self-coupling of the node's trace.
// ============================================================================
template <int N, bool MOM>
__global__ __launch_bounds__(256) void k_map_diag(MapMesh mm, Tables t, double fac, double mc,
                                                   double tnu, double th,
                                                   const double* __restrict__ w,
                                                   double* __restrict__ d, int Nc) {
    constexpr int NB = N * N;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (int64_t)Nc * NB) return;
    const int cell = (int)(gid / NB), nd = (int)(gid % NB);
    const int i0 = nd % N, i1 = nd / N;
    const double* D = MOM ? t.Du : t.Dp;
    const double* xr = MOM ? t.xu : t.xp;
    const double* Wr = MOM ? t.Wu : t.Wp;
    const double* L0 = MOM ? t.L0u : t.L0p;
    const double* L1 = MOM ? t.L1u : t.L1p;
    const double* dL0 = MOM ? t.dL0u : t.dL0p;
    const double* dL1 = MOM ? t.dL1u : t.dL1p;
    double X[8];
#pragma unroll
    for (int v = 0; v < 8; ++v) X[v] = mm.vtx[(size_t)cell * 8 + v];
    const double kap = MOM ? tnu : 1.0;
    double acc = 0.0;
    {
        const Adj J = map_adj(X, xr[i0], xr[i1]);
        const double W = Wr[i0] * Wr[i1];
        acc += mc * W * J.det;
        const double wd = W / J.det;
        const double P01 = J.m00 * J.m10 + J.m01 * J.m11;
        acc += kap * 2.0 * D[i0 * N + i0] * D[i1 * N + i1] * wd * P01;
        if (MOM) {
            const double w0 = w[((size_t)cell * 2) * NB + nd], w1 = w[((size_t)cell * 2 + 1) * NB + nd];
            const double c0 = W * (J.m00 * w0 + J.m01 * w1), c1 = W * (J.m10 * w0 + J.m11 * w1);
            acc -= th * (D[i0 * N + i0] * c0 + D[i1 * N + i1] * c1);
        }
    }
    for (int q = 0; q < N; ++q) {
        {
            const Adj J = map_adj(X, xr[q], xr[i1]);
            const double wd = Wr[q] * Wr[i1] / J.det;
            const double dq = D[q * N + i0];
            acc += kap * dq * dq * wd * (J.m00 * J.m00 + J.m01 * J.m01);
        }
        {
            const Adj J = map_adj(X, xr[i0], xr[q]);
            const double wd = Wr[i0] * Wr[q] / J.det;
            const double dq = D[q * N + i1];
            acc += kap * dq * dq * wd * (J.m10 * J.m10 + J.m11 * J.m11);
        }
    }
    for (int f = 0; f < 4; ++f) {
        const int a = f >> 1, s = f & 1;
        const int ia = a == 0 ? i0 : i1, ib = a == 0 ? i1 : i0;
        const double L = (s ? L1 : L0)[ia], dL = (s ? dL1 : dL0)[ia];
        const FaceG G = face_geo(X, a, s, xr[ib], Wr[ib]);
        const double ndv = G.va * dL + G.vb * L * D[ib * N + ib];
        const int nb = map_nbr(mm, cell, f);
        if (nb >= 0) {
            const double C = 0.5 * fac * (mm.gr[(size_t)cell * 4 + f] + mm.gr[(size_t)nb * 4 + (f ^ 1)]);
            acc += kap * G.dS * (-L * ndv + C * L * L);
            if (MOM) {
                const double* Ls = s ? t.L1u : t.L0u;
                const double* Ln = s ? t.L0u : t.L1u;
                double wK[2] = {0.0, 0.0}, wN[2] = {0.0, 0.0};
                for (int c = 0; c < 2; ++c)
                    for (int m = 0; m < N; ++m) {
                        const int ln = mnode<N>(a, m, ib);
                        wK[c] += Ls[m] * w[((size_t)cell * 2 + c) * NB + ln];
                        wN[c] += Ln[m] * w[((size_t)nb * 2 + c) * NB + ln];
                    }
                const double wnK = wK[0] * G.n0 + wK[1] * G.n1, wnN = wN[0] * G.n0 + wN[1] * G.n1;
                const double lam = fmax(fabs(wnK), fabs(wnN));
                acc += th * G.dS * L * L * 0.5 * (wnK + lam);
            }
        } else if (MOM) {
            const double C = fac * mm.gr[(size_t)cell * 4 + f];
            acc += kap * G.dS * (-2.0 * L * ndv + 2.0 * C * L * L);
            const double* Ls = s ? t.L1u : t.L0u;
            double wK[2] = {0.0, 0.0};
            for (int c = 0; c < 2; ++c)
                for (int m = 0; m < N; ++m) wK[c] += Ls[m] * w[((size_t)cell * 2 + c) * NB + mnode<N>(a, m, ib)];
            const int64_t pt = map_bnd_point(mm, cell, a, s, ib, N);
            const double e0 = 2.0 * mm.uD[pt * 2] - wK[0], e1 = 2.0 * mm.uD[pt * 2 + 1] - wK[1];
            const double lam = fmax(fabs(wK[0] * G.n0 + wK[1] * G.n1), fabs(e0 * G.n0 + e1 * G.n1));
            acc += th * G.dS * L * L * lam;
        }
    }
    d[gid] = acc;
}

// ============================================================================
// Explicit momentum right-hand side (eq. rhs1 and its stage-2 analogue):
// rhs = m M u_prev + sum_k [ -cd_k L0 u_k + ca_k A0(w_k) u_k ] + Gw p with
//   L0(u, v)   = int grad u . grad v - sum_E int {{grad u}} . [[v]],
//   A0_w(u, v) = int u (w . grad v) - sum_E int {{u w}} . [[v]],
//   Gw p (v)   = int p div v - sum_E int {{p}} [[v]]
// (no penalty, no upwinding; on a boundary face the average is the interior
// trace).  The volume fluxes and face values of the pairs and of p are
// accumulated per thread and contracted once at the end.
// ============================================================================
template <int N>
__global__ __launch_bounds__(256) void k_map_rhs(MapMesh mm, Tables t, double mc,
                                                  const double* __restrict__ u_prev,
                                                  const double* __restrict__ u1,
                                                  const double* __restrict__ w1, double cd1,
                                                  double ca1, const double* __restrict__ u2,
                                                  const double* __restrict__ w2, double cd2,
                                                  double ca2, const double* __restrict__ p,
                                                  double* __restrict__ rhs, int Nc) {
    constexpr int NB = N * N, CPB = mcpb(NB), NFP = 4 * N, NREC = CPB * NFP;
    constexpr int NP = N - 1, NBP = NP * NP;
    static_assert(NREC <= 256, "one face point per thread");
    __shared__ double s_X[CPB * 8];
    __shared__ double s_XN[CPB * 32];
    __shared__ int s_nb[CPB * 4];
    __shared__ double s_u[2][256];
    __shared__ double s_w[2][256];
    __shared__ double s_F[2][2][256];
    __shared__ double s_A[10][256];   // uK[2] dK[2] uN[2] dN[2] wnK wnN (w traces first)
    __shared__ double s_V[2][256];
    const int tid = threadIdx.x;
    const int lc = tid / NB, nd = tid % NB;
    const int cell0 = blockIdx.x * CPB;
    const int cell = cell0 + lc;
    const bool active = lc < CPB && cell < Nc;
    stage_geometry<CPB>(mm, cell0, Nc, s_X, s_XN, s_nb);
    const double* D = t.Du;
    const int q0 = nd % N, q1 = nd / N, base = lc * NB;
    Adj J{0, 0, 0, 0, 1};
    double W = 0.0;
    if (active) {
        J = map_adj(s_X + lc * 8, t.xu[q0], t.xu[q1]);
        W = t.Wu[q0] * t.Wu[q1];
    }
    double F[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
    double V[2] = {0.0, 0.0};
    const int lf = tid / NFP, f = (tid % NFP) / N, tt = tid % N;
    const int a = f >> 1, s = f & 1;
    const int fcell = cell0 + lf;
    const bool frec = tid < NREC && fcell < Nc;
    FaceG G{0, 0, 0, 0, 0};
    double va2 = 0.0, vb2 = 0.0;
    int fnb = -1;
    if (frec) {
        G = face_geo(s_X + lf * 8, a, s, t.xu[tt], t.Wu[tt]);
        fnb = s_nb[lf * 4 + f];
        if (fnb >= 0) nbr_ref(s_XN + (lf * 4 + f) * 8, a, s, t.xu[tt], G.n0, G.n1, va2, vb2);
    }
    for (int k = 0; k < 2; ++k) {
        const double* uk = k == 0 ? u1 : u2;
        const double* wk = k == 0 ? w1 : w2;
        const double cd = k == 0 ? cd1 : cd2, ca = k == 0 ? ca1 : ca2;
        if (!uk) continue;
        __syncthreads();   // previous pair's readers of s_u / s_A are done
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const size_t gi = ((size_t)cell * 2 + c) * NB + nd;
            s_u[c][tid] = active ? uk[gi] : 0.0;
            s_w[c][tid] = active ? wk[gi] : 0.0;
        }
        __syncthreads();
        if (active) {
            const double wd = W / J.det;
            const double P00 = J.m00 * J.m00 + J.m01 * J.m01, P01 = J.m00 * J.m10 + J.m01 * J.m11,
                         P11 = J.m10 * J.m10 + J.m11 * J.m11;
            const double w0 = s_w[0][tid], w1v = s_w[1][tid];
            const double c0 = W * (J.m00 * w0 + J.m01 * w1v), c1 = W * (J.m10 * w0 + J.m11 * w1v);
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                double g0 = 0.0, g1 = 0.0;
#pragma unroll
                for (int j = 0; j < N; ++j) {
                    g0 += D[q0 * N + j] * s_u[c][base + j + N * q1];
                    g1 += D[q1 * N + j] * s_u[c][base + q0 + N * j];
                }
                const double uq = s_u[c][tid];
                F[c][0] += -cd * wd * (P00 * g0 + P01 * g1) + ca * uq * c0;
                F[c][1] += -cd * wd * (P01 * g0 + P11 * g1) + ca * uq * c1;
            }
        }
        if (frec) {
            const double* Ls = s ? t.L1u : t.L0u;
            const double* dLs = s ? t.dL1u : t.dL0u;
            const double* Ln = s ? t.L0u : t.L1u;
            const double* dLn = s ? t.dL0u : t.dL1u;
            double wK[2] = {0.0, 0.0}, wN[2] = {0.0, 0.0};
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                double uK = 0.0, dK = 0.0, uN = 0.0, dN = 0.0;
#pragma unroll
                for (int m = 0; m < N; ++m) {
                    const int li = lf * NB + mnode<N>(a, m, tt);
                    uK += Ls[m] * s_u[c][li];
                    dK += dLs[m] * s_u[c][li];
                    wK[c] += Ls[m] * s_w[c][li];
                }
                if (fnb >= 0) {
#pragma unroll
                    for (int m = 0; m < N; ++m) {
                        const size_t gi = ((size_t)fnb * 2 + c) * NB + mnode<N>(a, m, tt);
                        const double v = uk[gi];
                        uN += Ln[m] * v;
                        dN += dLn[m] * v;
                        wN[c] += Ln[m] * wk[gi];
                    }
                }
                s_A[0 + c][tid] = uK;
                s_A[2 + c][tid] = dK;
                s_A[4 + c][tid] = uN;
                s_A[6 + c][tid] = dN;
            }
            s_A[8][tid] = wK[0] * G.n0 + wK[1] * G.n1;
            s_A[9][tid] = wN[0] * G.n0 + wN[1] * G.n1;
        }
        __syncthreads();
        if (frec) {
            const int rb = lf * NFP + f * N;
            const double wnK = s_A[8][tid], wnN = s_A[9][tid];
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                double tK = 0.0, tN = 0.0;
#pragma unroll
                for (int j = 0; j < N; ++j) {
                    tK += D[tt * N + j] * s_A[0 + c][rb + j];
                    tN += D[tt * N + j] * s_A[4 + c][rb + j];
                }
                const double uK = s_A[0 + c][tid], uN = s_A[4 + c][tid];
                const double ndK = G.va * s_A[2 + c][tid] + G.vb * tK;
                if (fnb >= 0) {
                    const double ndN = va2 * s_A[6 + c][tid] + vb2 * tN;
                    V[c] += G.dS * (cd * 0.5 * (ndK - ndN) - ca * 0.5 * (wnK * uK + wnN * uN));
                } else {
                    V[c] += G.dS * (cd * ndK - ca * wnK * uK);
                }
            }
        }
    }
    // weak gradient of p: volume p (adj)^T e_c, faces -{{p}} n_c
    if (p) {
        __syncthreads();
        for (int it = tid; it < CPB * NBP; it += 256) {
            const int c2 = cell0 + it / NBP;
            s_u[0][it] = c2 < Nc ? p[(size_t)c2 * NBP + it % NBP] : 0.0;
        }
        __syncthreads();
        if (active) {
            double pq = 0.0;
            for (int j = 0; j < NBP; ++j)
                pq += t.Ip[q0 * NMAX + j % NP] * t.Ip[q1 * NMAX + j / NP] * s_u[0][lc * NBP + j];
            // (G grad_xi v)_c det = sum_b adj[b][c] d_b v
            F[0][0] += W * pq * J.m00;
            F[0][1] += W * pq * J.m10;
            F[1][0] += W * pq * J.m01;
            F[1][1] += W * pq * J.m11;
        }
        if (frec) {
            const double* Lps = s ? t.L1p : t.L0p;
            const double* Lpn = s ? t.L0p : t.L1p;
            double pK = 0.0, pN = 0.0;
            for (int j = 0; j < NBP; ++j) {
                const int ja = a == 0 ? j % NP : j / NP, jb = a == 0 ? j / NP : j % NP;
                const double bK = Lps[ja] * t.Ip[tt * NMAX + jb];
                pK += bK * s_u[0][lf * NBP + j];
                if (fnb >= 0) pN += Lpn[ja] * t.Ip[tt * NMAX + jb] * p[(size_t)fnb * NBP + j];
            }
            const double pa = fnb >= 0 ? 0.5 * (pK + pN) : pK;
            V[0] -= G.dS * pa * G.n0;
            V[1] -= G.dS * pa * G.n1;
        }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        s_F[c][0][tid] = F[c][0];
        s_F[c][1][tid] = F[c][1];
        s_V[c][tid] = V[c];
    }
    __syncthreads();
    if (active) {
        const int i0 = q0, i1 = q1;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const size_t gi = ((size_t)cell * 2 + c) * NB + nd;
            double acc = mc * W * J.det * u_prev[gi];
#pragma unroll
            for (int q = 0; q < N; ++q)
                acc += D[q * N + i0] * s_F[c][0][base + q + N * i1] +
                       D[q * N + i1] * s_F[c][1][base + i0 + N * q];
#pragma unroll
            for (int ff = 0; ff < 4; ++ff) {
                const int aa = ff >> 1, ss = ff & 1;
                const int ia = aa == 0 ? i0 : i1, ib = aa == 0 ? i1 : i0;
                acc += (ss ? t.L1u : t.L0u)[ia] * s_V[c][lc * NFP + ff * N + ib];
            }
            rhs[gi] = acc;
        }
    }
}

// Dirichlet-data terms of stage s on the boundary faces normal to direction a
// (the boundary part of eq. rhs1): for each component c
//   -theta nu int u_D,c (n . grad v) + theta nu int 2 C u_D,c v
//   - theta int u_D,c (w . n) v + theta int lambda u_D,c v,
// lambda = max(|w . n|, |(2 u_D - w) . n|).  One thread per (boundary cell,
// node, component) accumulates both sides of its cell.
template <int N>
__global__ __launch_bounds__(256) void k_map_dirichlet(MapMesh mm, Tables t, int a, double fac,
                                                        double tnu, double th,
                                                        const double* __restrict__ w,
                                                        double* __restrict__ rhs) {
    constexpr int NB = N * N;
    const int ncf = mm.nc[1 - a];
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (int64_t)ncf * NB * 2) return;
    const int c = (int)(gid % 2);
    const int nd = (int)((gid / 2) % NB);
    const int tc = (int)(gid / (2 * NB));
    const int i0 = nd % N, i1 = nd / N;
    const int ia = a == 0 ? i0 : i1, ib = a == 0 ? i1 : i0;
    double acc_by_side[2] = {0.0, 0.0};
    int cells[2];
    for (int s = 0; s < 2; ++s) {
        const int ca = s ? mm.nc[a] - 1 : 0;
        const int cell = a == 0 ? ca + mm.nc[0] * tc : tc + mm.nc[0] * ca;
        cells[s] = cell;
        double X[8];
#pragma unroll
        for (int v = 0; v < 8; ++v) X[v] = mm.vtx[(size_t)cell * 8 + v];
        const double* Ls = s ? t.L1u : t.L0u;
        const double L = Ls[ia], dL = (s ? t.dL1u : t.dL0u)[ia];
        const double C = fac * mm.gr[(size_t)cell * 4 + 2 * a + s];
        double acc = 0.0;
        for (int q = 0; q < N; ++q) {
            const FaceG G = face_geo(X, a, s, t.xu[q], t.Wu[q]);
            const int64_t pt = mm.off[a][s] + (int64_t)tc * N + q;
            double wK[2] = {0.0, 0.0};
            for (int cc = 0; cc < 2; ++cc)
                for (int m = 0; m < N; ++m) wK[cc] += Ls[m] * w[((size_t)cell * 2 + cc) * NB + mnode<N>(a, m, q)];
            const double wn = wK[0] * G.n0 + wK[1] * G.n1;
            const double e0 = 2.0 * mm.uD[pt * 2] - wK[0], e1 = 2.0 * mm.uD[pt * 2 + 1] - wK[1];
            const double lam = fmax(fabs(wn), fabs(e0 * G.n0 + e1 * G.n1));
            const double g = mm.uD[pt * 2 + c] * G.dS;
            // grad v . n at this point: va dL delta(ib, q) + vb L D[q][ib]
            double gn = G.vb * L * t.Du[q * N + ib];
            double val = 0.0;
            if (q == ib) {
                gn += G.va * dL;
                val = (tnu * 2.0 * C - th * wn + th * lam) * L;
            }
            acc += g * (-tnu * gn + val);
        }
        acc_by_side[s] = acc;
    }
    if (cells[0] == cells[1]) {
        rhs[((size_t)cells[0] * 2 + c) * NB + nd] += acc_by_side[0] + acc_by_side[1];
    } else {
        rhs[((size_t)cells[0] * 2 + c) * NB + nd] += acc_by_side[0];
        rhs[((size_t)cells[1] * 2 + c) * NB + nd] += acc_by_side[1];
    }
}

// ============================================================================
// Helmholtz right-hand side alpha M^p p_prev + fcoef D u** with
// D u (q) = int u . grad q - sum_E int {{u}} . [[q]] (velocity rule; the
// average is the interior trace on a boundary face).
// ============================================================================
template <int N>
__global__ __launch_bounds__(256) void k_map_rhs_p(MapMesh mm, Tables t, double alpha, double fcoef,
                                                    const double* __restrict__ uss,
                                                    const double* __restrict__ p_prev,
                                                    double* __restrict__ rhs, int Nc) {
    constexpr int NB = N * N, CPB = mcpb(NB), NFP = 4 * N, NREC = CPB * NFP;
    constexpr int NP = N - 1, NBP = NP * NP;
    static_assert(NREC <= 256, "one face point per thread");
    __shared__ double s_X[CPB * 8];
    __shared__ int s_nb[CPB * 4];
    __shared__ double s_u[2][256];
    __shared__ double s_F[2][256];
    __shared__ double s_B[256];
    const int tid = threadIdx.x;
    const int lc = tid / NB, nd = tid % NB;
    const int cell0 = blockIdx.x * CPB;
    const int cell = cell0 + lc;
    const bool active = lc < CPB && cell < Nc;
#pragma unroll
    for (int c = 0; c < 2; ++c) s_u[c][tid] = active ? uss[((size_t)cell * 2 + c) * NB + nd] : 0.0;
    stage_geometry<CPB>(mm, cell0, Nc, s_X, nullptr, s_nb);
    if (active) {
        const int q0 = nd % N, q1 = nd / N;
        const Adj J = map_adj(s_X + lc * 8, t.xu[q0], t.xu[q1]);
        const double W = t.Wu[q0] * t.Wu[q1];
        const double u0 = s_u[0][tid], u1 = s_u[1][tid];
        s_F[0][tid] = W * (J.m00 * u0 + J.m01 * u1);
        s_F[1][tid] = W * (J.m10 * u0 + J.m11 * u1);
    }
    const int lf = tid / NFP, f = (tid % NFP) / N, tt = tid % N;
    const int a = f >> 1, s = f & 1;
    if (tid < NREC && cell0 + lf < Nc) {
        const double* Ls = s ? t.L1u : t.L0u;
        const double* Ln = s ? t.L0u : t.L1u;
        const int nb = s_nb[lf * 4 + f];
        double uf[2];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            double uK = 0.0, uN = 0.0;
#pragma unroll
            for (int m = 0; m < N; ++m) {
                uK += Ls[m] * s_u[c][lf * NB + mnode<N>(a, m, tt)];
                if (nb >= 0) uN += Ln[m] * uss[((size_t)nb * 2 + c) * NB + mnode<N>(a, m, tt)];
            }
            uf[c] = nb >= 0 ? 0.5 * (uK + uN) : uK;
        }
        const FaceG G = face_geo(s_X + lf * 8, a, s, t.xu[tt], t.Wu[tt]);
        s_B[tid] = G.dS * (uf[0] * G.n0 + uf[1] * G.n1);
    }
    __syncthreads();
    if (lc < CPB && cell < Nc && nd < NBP) {
        const int i0 = nd % NP, i1 = nd / NP;
        double acc = 0.0;
        for (int q = 0; q < NB; ++q) {
            const int r0 = q % N, r1 = q / N;
            acc += t.Dpu[r0 * NMAX + i0] * t.Ip[r1 * NMAX + i1] * s_F[0][lc * NB + q] +
                   t.Ip[r0 * NMAX + i0] * t.Dpu[r1 * NMAX + i1] * s_F[1][lc * NB + q];
        }
        for (int ff = 0; ff < 4; ++ff) {
            const int aa = ff >> 1, ss = ff & 1;
            const int ia = aa == 0 ? i0 : i1, ib = aa == 0 ? i1 : i0;
            const double Lp = (ss ? t.L1p : t.L0p)[ia];
            double g = 0.0;
            for (int q = 0; q < N; ++q) g += t.Ip[q * NMAX + ib] * s_B[lc * NFP + ff * N + q];
            acc -= Lp * g;
        }
        const Adj J = map_adj(s_X + lc * 8, t.xp[i0], t.xp[i1]);
        const size_t gi = (size_t)cell * NBP + nd;
        rhs[gi] = alpha * t.Wp[i0] * t.Wp[i1] * J.det * p_prev[gi] + fcoef * acc;
    }
}

// y = x + a grad p at the velocity nodes (M^{-1} P p: the projection matrix
// with the collocated diagonal velocity mass gives the nodal gradient).
template <int N>
__global__ __launch_bounds__(256) void k_map_grad_p(MapMesh mm, Tables t, const double* x, double a,
                                                     const double* __restrict__ p, double* y,
                                                     int Nc) {
    constexpr int NB = N * N, NP = N - 1, NBP = NP * NP;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (int64_t)Nc * NB) return;
    const int cell = (int)(gid / NB), nd = (int)(gid % NB);
    const int i0 = nd % N, i1 = nd / N;
    const double* pc = p + (size_t)cell * NBP;
    double g0 = 0.0, g1 = 0.0;
    for (int j = 0; j < NBP; ++j) {
        const int j0 = j % NP, j1 = j / NP;
        g0 += t.Dpu[i0 * NMAX + j0] * t.Ip[i1 * NMAX + j1] * pc[j];
        g1 += t.Ip[i0 * NMAX + j0] * t.Dpu[i1 * NMAX + j1] * pc[j];
    }
    const Adj J = map_adj(mm.vtx + (size_t)cell * 8, t.xu[i0], t.xu[i1]);
    const double gr[2] = {(J.m00 * g0 + J.m10 * g1) / J.det, (J.m01 * g0 + J.m11 * g1) / J.det};
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const size_t idx = ((size_t)cell * 2 + c) * NB + nd;
        const double xv = x ? x[idx] : 0.0;
        y[idx] = xv + a * gr[c];
    }
}

// physical node coordinates [cell][node][2]
__global__ void k_map_coords(MapMesh mm, Tables t, int field, int n, double* xyz, int Nc) {
    const int nb = n * n;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (int64_t)Nc * nb) return;
    const int cell = (int)(gid / nb), nd = (int)(gid % nb);
    const double* xr = field == 0 ? t.xu : t.xp;
    const double x0 = xr[nd % n], x1 = xr[nd / n];
    const double* X = mm.vtx + (size_t)cell * 8;
    const double b0 = (1.0 - x0) * (1.0 - x1), b1 = x0 * (1.0 - x1), b2 = (1.0 - x0) * x1, b3 = x0 * x1;
    xyz[gid * 2] = b0 * X[0] + b1 * X[2] + b2 * X[4] + b3 * X[6];
    xyz[gid * 2 + 1] = b0 * X[1] + b1 * X[3] + b2 * X[5] + b3 * X[7];
}

inline unsigned nblk(int64_t work, int per) { return (unsigned)((work + per - 1) / per); }

}  // namespace

// ---------------------------------------------------------------------------
#define TBDG_MAP_DISPATCH(n, FN)                                                          \
    do {                                                                                  \
        if ((n) == 3) { FN(3); }                                                          \
        else if ((n) == 4) { FN(4); }                                                     \
        else if ((n) == 5) { FN(5); }                                                     \
        else if ((n) == 6) { FN(6); }                                                     \
        else throw Error(TBDG_EUNSUPPORTED, "unsupported degree on mapped cells");        \
    } while (0)
#define TBDG_MAP_DISPATCH_P(n, FN)                                                        \
    do {                                                                                  \
        if ((n) == 2) { FN(2); }                                                          \
        else if ((n) == 3) { FN(3); }                                                     \
        else if ((n) == 4) { FN(4); }                                                     \
        else if ((n) == 5) { FN(5); }                                                     \
        else throw Error(TBDG_EUNSUPPORTED, "unsupported degree on mapped cells");        \
    } while (0)

MapMesh map_mesh(const tbdg_ctx* c, int s) {
    MapMesh m{};
    m.vtx = c->map_vtx;
    m.gr = c->map_gr;
    m.nc[0] = c->geom.nc[0];
    m.nc[1] = c->geom.nc[1];
    m.per[0] = c->periodic_flags[0];
    m.per[1] = c->periodic_flags[1];
    for (int a = 0; a < 2; ++a)
        for (int k = 0; k < 2; ++k) m.off[a][k] = c->bnd_off[a][k];
    m.uD = c->bnd_uD[c->bnd_slot(s)];
    return m;
}

static double fac_u(const tbdg_ctx* c) { return (c->k + 1.0) * (c->k + 1.0) * c->pen_u; }
static double fac_p(const tbdg_ctx* c) { return (double)c->k * c->k * c->pen_p; }

void map_apply_pressure(const tbdg_ctx* c, double alpha, const double* p, double* y, int mode,
                        double* partial, const double* r, const double* invd, double* sc,
                        double* p_out, const double* up, int Gu, int first, int slot,
                        int slot_prev, int* G_out) {
    const MapMesh mm = map_mesh(c, 1);
    const double bytes = (mode == 0 ? 16.0 : mode == 3 ? 40.0 : 32.0) * (double)c->Np;
#define L_(NP)                                                                            \
    {                                                                                     \
        constexpr int CPB = mcpb(NP * NP);                                                \
        const int G = (int)nblk(c->Nc, CPB);                                              \
        if (mode >= 3 && G > c->red_op_len) throw Error(TBDG_EINVAL, "operator partial buffer too small"); \
        if (G_out) *G_out = G;                                                            \
        TimedLaunch tl(c, 0, bytes);                                                      \
        if (mode == 0)                                                                    \
            hipExtLaunchKernelGGL((k_map_pres<NP, 0>), dim3(G), dim3(256), 0, c->stream,  \
                                  tl.start(), tl.stop(), 0, mm, c->tab, fac_p(c), alpha, p, y, \
                                  (int)c->Nc, partial, r, invd, sc, p_out, up, Gu, first, slot, \
                                  slot_prev);                                             \
        else if (mode == 3)                                                               \
            hipExtLaunchKernelGGL((k_map_pres<NP, 3>), dim3(G), dim3(256), 0, c->stream,  \
                                  tl.start(), tl.stop(), 0, mm, c->tab, fac_p(c), alpha, p, y, \
                                  (int)c->Nc, partial, r, invd, sc, p_out, up, Gu, first, slot, \
                                  slot_prev);                                             \
        else                                                                              \
            hipExtLaunchKernelGGL((k_map_pres<NP, 4>), dim3(G), dim3(256), 0, c->stream,  \
                                  tl.start(), tl.stop(), 0, mm, c->tab, fac_p(c), alpha, p, y, \
                                  (int)c->Nc, partial, r, invd, sc, p_out, up, Gu, first, slot, \
                                  slot_prev);                                             \
    }
    TBDG_MAP_DISPATCH_P(c->np, L_);
#undef L_
    TBDG_HIP(hipGetLastError());
}

void map_diag_pressure(const tbdg_ctx* c, double alpha, double* d) {
    const MapMesh mm = map_mesh(c, 1);
#define L_(NP)                                                                            \
    hipLaunchKernelGGL((k_map_diag<NP, false>), dim3(nblk(c->Np, 256)), dim3(256), 0,     \
                       c->stream, mm, c->tab, fac_p(c), alpha, 0.0, 0.0, nullptr, d,      \
                       (int)c->Nc);
    TBDG_MAP_DISPATCH_P(c->np, L_);
#undef L_
    TBDG_HIP(hipGetLastError());
}

int map_apply_momentum(const tbdg_ctx* c, int st, const double* w, const double* u, double* y,
                       const MomFuse& fz) {
    const MapMesh mm = map_mesh(c, st);
    double bytes = 24.0 * (double)c->Nu;
    if (fz.invd) bytes += 8.0 * (double)c->Ns;
    if (fz.shv) bytes += 8.0 * (double)c->Nu;
    bytes += 8.0 * fz.ndot * (double)c->Nu;
    int G = 0;
#define L_(N)                                                                             \
    {                                                                                     \
        constexpr int CPB = mcpb(N * N);                                                  \
        G = (int)nblk(c->Nc, CPB);                                                        \
        if (fz.ndot > 0 && (int64_t)G * (fz.ndot + 1) > c->gm_part_len)                   \
            throw Error(TBDG_EINVAL, "fused partial buffer too small");                   \
        TimedLaunch tl(c, 1, bytes);                                                      \
        hipExtLaunchKernelGGL((k_map_mom<N>), dim3(G), dim3(256), 0, c->stream, tl.start(), \
                              tl.stop(), 0, mm, c->tab, fac_u(c), c->mcoef(st),           \
                              c->theta[st] * c->nu, c->theta[st], w, u, y, (int)c->Nc, fz); \
    }
    TBDG_MAP_DISPATCH(c->n, L_);
#undef L_
    TBDG_HIP(hipGetLastError());
    return G;
}

void map_diag_momentum(const tbdg_ctx* c, int st, const double* w, double* d) {
    const MapMesh mm = map_mesh(c, st);
#define L_(N)                                                                             \
    hipLaunchKernelGGL((k_map_diag<N, true>), dim3(nblk(c->Ns, 256)), dim3(256), 0,       \
                       c->stream, mm, c->tab, fac_u(c), c->mcoef(st), c->theta[st] * c->nu, \
                       c->theta[st], w, d, (int)c->Nc);
    TBDG_MAP_DISPATCH(c->n, L_);
#undef L_
    TBDG_HIP(hipGetLastError());
}

void map_rhs_momentum(const tbdg_ctx* c, double mcoef, const double* u_prev, const double* u1,
                      const double* w1, double cd1, double ca1, const double* u2, const double* w2,
                      double cd2, double ca2, const double* p, double* rhs) {
    const MapMesh mm = map_mesh(c, 1);
#define L_(N)                                                                             \
    hipLaunchKernelGGL((k_map_rhs<N>), dim3(nblk(c->Nc, mcpb(N * N))), dim3(256), 0,      \
                       c->stream, mm, c->tab, mcoef, u_prev, u1, w1, cd1, ca1, u2, w2, cd2, \
                       ca2, p, rhs, (int)c->Nc);
    TBDG_MAP_DISPATCH(c->n, L_);
#undef L_
    TBDG_HIP(hipGetLastError());
}

void map_dirichlet_rhs(const tbdg_ctx* c, int s, const double* w, double* rhs) {
    const MapMesh mm = map_mesh(c, s);
    for (int a = 0; a < 2; ++a) {
        if (mm.off[a][0] < 0) continue;
        const int64_t work = (int64_t)mm.nc[1 - a] * c->nbu * 2;
#define L_(N)                                                                             \
        hipLaunchKernelGGL((k_map_dirichlet<N>), dim3(nblk(work, 256)), dim3(256), 0,     \
                           c->stream, mm, c->tab, a, fac_u(c), c->theta[s] * c->nu,       \
                           c->theta[s], w, rhs);
        TBDG_MAP_DISPATCH(c->n, L_);
#undef L_
        TBDG_HIP(hipGetLastError());
    }
}

void map_rhs_pressure(const tbdg_ctx* c, double alpha, double fcoef, const double* u_ss,
                      const double* p_prev, double* rhs) {
    const MapMesh mm = map_mesh(c, 1);
#define L_(N)                                                                             \
    hipLaunchKernelGGL((k_map_rhs_p<N>), dim3(nblk(c->Nc, mcpb(N * N))), dim3(256), 0,    \
                       c->stream, mm, c->tab, alpha, fcoef, u_ss, p_prev, rhs, (int)c->Nc);
    TBDG_MAP_DISPATCH(c->n, L_);
#undef L_
    TBDG_HIP(hipGetLastError());
}

void map_add_grad_p(const tbdg_ctx* c, const double* x, double a, const double* p, double* y) {
    const MapMesh mm = map_mesh(c, 1);
#define L_(N)                                                                             \
    hipLaunchKernelGGL((k_map_grad_p<N>), dim3(nblk(c->Ns, 256)), dim3(256), 0, c->stream, \
                       mm, c->tab, x, a, p, y, (int)c->Nc);
    TBDG_MAP_DISPATCH(c->n, L_);
#undef L_
    TBDG_HIP(hipGetLastError());
}

void map_node_coords(const tbdg_ctx* c, int field, double* xyz) {
    const MapMesh mm = map_mesh(c, 1);
    const int n = field == 0 ? c->n : c->np;
    const int64_t work = c->Nc * (int64_t)n * n;
    hipLaunchKernelGGL(k_map_coords, dim3(nblk(work, 256)), dim3(256), 0, c->stream, mm, c->tab,
                       field, n, xyz, (int)c->Nc);
    TBDG_HIP(hipGetLastError());
}

}  // namespace trbdg
