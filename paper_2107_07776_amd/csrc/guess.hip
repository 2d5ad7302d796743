// Cell-grid inputs and outputs of the learned pressure initial guess.
//
// Per Helmholtz solve of stage s (beta_s, right-hand side b, previous
// pressure p) with the same stage's increments d1, d2 of the last two steps
// and the newest increment d0 (weight beta0), <a, c>_K = sum_{i in K} W_i a_i c_i
// (W_i: product of the Gauss weights of node i on the unit cell):
//   m1_K = <d1, 1>_K / (beta_s dt),  m2_K = <d2, 1>_K / (beta_s dt),
//   m0_K = <d0, 1>_K / (beta0 dt),
//   div_K = -(beta_s dt / |K|) sum_{i in K} (b_i - alpha |K| W_i p_i),
//   cos_K = <d1, d2>_K / sqrt(<d1, d1>_K <d2, d2>_K),
//   lr_K = clamp(log(<d1, d1>_K / <d2, d2>_K) / 2, -4, 4)   (0 without history);
// network input (m1 / s_inc, m2 / s_inc, m0 / s_inc, div / s_div, cos, lr)
// with s_inc, s_div the RMS over cells of m1 and div (1 where zero).  The
// network output (y0_K, y1_K) corrects the blend of the increments: the
// guess is p + (2 + y0_K) d1 - (1 - y1_K) d2 at the nodes of K (y = 0: the
// increment extrapolated from its last two values).  Training target per
// cell: the Gram data (<d1,d1>, <d1,d2>, <d2,d2>, <e,d1>, <e,d2>, <e,e>)_K / S
// of the extrapolation's error e = p_new - (p + 2 d1 - d2), S the mean over
// cells of <d1,d1>_K.
#include <hip/hip_runtime.h>

#include "internal.hpp"
#include "reduce.hpp"

namespace trbdg {
namespace {

constexpr int ipw(int b, int e) { return e == 0 ? 1 : b * ipw(b, e - 1); }

template <int DIM, int NP>
__device__ inline double node_weight(const double* W, int i) {
    double w = 1.0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        w *= W[i % NP];
        i /= NP;
    }
    return w;
}

// Cells of a block: one thread per node loads it (coalesced) and forms its
// weighted terms, one thread per cell sums them in node order.
template <int DIM, int NP>
struct CellBlock {
    static constexpr int NB = ipw(NP, DIM);
    static constexpr int CPB = 256 / NB;
};

// m1, m2, m0, div, <d1,d1>, <d1,d2>, <d2,d2> into cells[7][Nc]; per-block
// partial sums of m1^2 and div^2
template <int DIM, int NP>
__global__ __launch_bounds__(256) void k_guess_cells(int Nc, Tables t, const double* __restrict__ d1,
                                                      const double* __restrict__ d2,
                                                      const double* __restrict__ d0,
                                                      const double* __restrict__ b,
                                                      const double* __restrict__ p, double c1, double c0,
                                                      double cdiv, double inv_vol, double alpha,
                                                      double* __restrict__ cells, double* partial) {
    using CB = CellBlock<DIM, NP>;
    constexpr int NB = CB::NB, CPB = CB::CPB;
    __shared__ double s_v[7][CPB * NB];
    const int tid = threadIdx.x;
    const int lc = tid / NB, nd = tid % NB;
    const int c = blockIdx.x * CPB + lc;
    if (lc < CPB) {
        double v[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        if (c < Nc) {
            const double w = node_weight<DIM, NP>(t.Wp, nd);
            const size_t gi = (size_t)c * NB + nd;
            const double a1 = d1[gi], a2 = d2[gi];
            v[0] = w * a1;
            v[1] = w * a2;
            v[2] = w * d0[gi];
            v[3] = b[gi] * inv_vol - alpha * w * p[gi];
            v[4] = w * a1 * a1;
            v[5] = w * a1 * a2;
            v[6] = w * a2 * a2;
        }
#pragma unroll
        for (int q = 0; q < 7; ++q) s_v[q][tid] = v[q];
    }
    __syncthreads();
    double m1 = 0.0, dv = 0.0;
    const int cc = blockIdx.x * CPB + tid;
    if (tid < CPB && cc < Nc) {
        double sum[7];
#pragma unroll
        for (int q = 0; q < 7; ++q) {
            double a = 0.0;
            for (int i = 0; i < NB; ++i) a += s_v[q][tid * NB + i];
            sum[q] = a;
        }
        m1 = sum[0] * c1;
        dv = sum[3] * cdiv;
        cells[cc] = m1;
        cells[Nc + cc] = sum[1] * c1;
        cells[2 * Nc + cc] = sum[2] * c0;
        cells[3 * Nc + cc] = dv;
        cells[4 * Nc + cc] = sum[4];
        cells[5 * Nc + cc] = sum[5];
        cells[6 * Nc + cc] = sum[6];
    }
    const double s0 = red::block_sum(m1 * m1);
    const double s2 = red::block_sum(dv * dv);
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = s0;
        partial[gridDim.x + blockIdx.x] = s2;
    }
}

// scales from the partials (every block sums them in the same order) and the
// FP32 network input [6][Nc]; block 0 stores (s_inc, s_div) in sc
__global__ __launch_bounds__(256) void k_guess_feat(int Nc, const double* __restrict__ cells,
                                                     const double* __restrict__ partial, int G,
                                                     float* __restrict__ feat, double* sc) {
    __shared__ double s_scale[2];
    double a = 0.0, d = 0.0;
    for (int k = threadIdx.x; k < G; k += 256) {
        a += partial[k];
        d += partial[G + k];
    }
    a = red::block_sum(a);
    d = red::block_sum(d);
    if (threadIdx.x == 0) {
        const double si = sqrt(a / Nc), sd = sqrt(d / Nc);
        s_scale[0] = si > 0.0 ? si : 1.0;
        s_scale[1] = sd > 0.0 ? sd : 1.0;
        if (blockIdx.x == 0) {
            sc[0] = s_scale[0];
            sc[1] = s_scale[1];
        }
    }
    __syncthreads();
    const double ri = 1.0 / s_scale[0], rd = 1.0 / s_scale[1];
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c < Nc) {
        const double g11 = cells[4 * Nc + c], g12 = cells[5 * Nc + c], g22 = cells[6 * Nc + c];
        double cs = 0.0, lr = 0.0;
        if (g11 > 0.0 && g22 > 0.0) {
            cs = g12 / sqrt(g11 * g22);
            lr = fmin(fmax(0.5 * log(g11 / g22), -4.0), 4.0);
        }
        feat[c] = (float)(cells[c] * ri);
        feat[Nc + c] = (float)(cells[Nc + c] * ri);
        feat[2 * Nc + c] = (float)(cells[2 * Nc + c] * ri);
        feat[3 * Nc + c] = (float)(cells[3 * Nc + c] * rd);
        feat[4 * Nc + c] = (float)cs;
        feat[5 * Nc + c] = (float)lr;
    }
}

// out_i = p_i + (2 + y0_K) d1_i - (1 - y1_K) d2_i, y = [2][Nc]
template <int NB>
__global__ __launch_bounds__(256) void k_guess_inject(int Nc, const double* __restrict__ p,
                                                       const double* __restrict__ d1,
                                                       const double* __restrict__ d2,
                                                       const double* __restrict__ d3,
                                                       const float* __restrict__ y,
                                                       double* __restrict__ out) {
    const int64_t n = (int64_t)Nc * NB;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const int c = (int)(i / NB);
        out[i] = p[i] + (3.0 + (double)y[c]) * d1[i] - (3.0 - (double)y[Nc + c]) * d2[i] + d3[i];
    }
}

// Gram data per cell into rows[6][Nc] (unscaled) and per-block partial sums
// of <d1,d1>_K
template <int DIM, int NP>
__global__ __launch_bounds__(256) void k_guess_gram(int Nc, Tables t, const double* __restrict__ pn,
                                                     const double* __restrict__ p,
                                                     const double* __restrict__ d1,
                                                     const double* __restrict__ d2,
                                                     const double* __restrict__ d3,
                                                     double* __restrict__ rows, double* partial) {
    using CB = CellBlock<DIM, NP>;
    constexpr int NB = CB::NB, CPB = CB::CPB;
    __shared__ double s_v[6][CPB * NB];
    const int tid = threadIdx.x;
    const int lc = tid / NB, nd = tid % NB;
    const int c = blockIdx.x * CPB + lc;
    if (lc < CPB) {
        double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        if (c < Nc) {
            const double w = node_weight<DIM, NP>(t.Wp, nd);
            const size_t gi = (size_t)c * NB + nd;
            const double a1 = d1[gi], a2 = d2[gi];
            const double e = pn[gi] - (p[gi] + 3.0 * a1 - 3.0 * a2 + d3[gi]);
            v[0] = w * a1 * a1;
            v[1] = w * a1 * a2;
            v[2] = w * a2 * a2;
            v[3] = w * e * a1;
            v[4] = w * e * a2;
            v[5] = w * e * e;
        }
#pragma unroll
        for (int q = 0; q < 6; ++q) s_v[q][tid] = v[q];
    }
    __syncthreads();
    double g11 = 0.0;
    const int cc = blockIdx.x * CPB + tid;
    if (tid < CPB && cc < Nc) {
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            double a = 0.0;
            for (int i = 0; i < NB; ++i) a += s_v[q][tid * NB + i];
            rows[(size_t)q * Nc + cc] = a;
            if (q == 0) g11 = a;
        }
    }
    const double s = red::block_sum(g11);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// out[6][Nc] = rows / S, S = mean over cells of <d1,d1>_K (1 where zero);
// every block sums the partials in the same order
__global__ __launch_bounds__(256) void k_guess_gram_scale(int Nc, const double* __restrict__ rows,
                                                           const double* __restrict__ partial, int G,
                                                           float* __restrict__ out) {
    __shared__ double s_inv;
    double a = 0.0;
    for (int k = threadIdx.x; k < G; k += 256) a += partial[k];
    a = red::block_sum(a);
    if (threadIdx.x == 0) {
        const double S = a / Nc;
        s_inv = S > 0.0 ? 1.0 / S : 1.0;
    }
    __syncthreads();
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c < Nc) {
#pragma unroll
        for (int r = 0; r < 6; ++r) out[(size_t)r * Nc + c] = (float)(rows[(size_t)r * Nc + c] * s_inv);
    }
}

inline unsigned nb256(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

#define TBDG_GUESS_DISPATCH(dim, np, FN)                                                  \
    do {                                                                                  \
        if ((dim) == 2 && (np) == 2) { FN(2, 2); }                                        \
        else if ((dim) == 2 && (np) == 3) { FN(2, 3); }                                   \
        else if ((dim) == 2 && (np) == 4) { FN(2, 4); }                                   \
        else if ((dim) == 2 && (np) == 5) { FN(2, 5); }                                   \
        else if ((dim) == 3 && (np) == 2) { FN(3, 2); }                                   \
        else if ((dim) == 3 && (np) == 3) { FN(3, 3); }                                   \
        else throw Error(TBDG_EUNSUPPORTED, "unsupported (dim, pressure nodes)");          \
    } while (0)

int launch_guess_cells(const tbdg_ctx* c, const double* d1, const double* d2, const double* d0,
                       const double* b, const double* p, double c1, double c0, double cdiv,
                       double alpha, double* cells, double* partial) {
    if (c->mapped)
        throw Error(TBDG_EUNSUPPORTED, "the learned guess is built for affine cells only");
    unsigned G = 0;
#define L_(D, NP)                                                                          \
    G = (unsigned)((c->Nc + CellBlock<D, NP>::CPB - 1) / CellBlock<D, NP>::CPB);           \
    hipLaunchKernelGGL((k_guess_cells<D, NP>), dim3(G), dim3(256), 0, c->stream, (int)c->Nc,  \
                       c->tab, d1, d2, d0, b, p, c1, c0, cdiv, 1.0 / c->geom.vol, alpha,   \
                       cells, partial);
    TBDG_GUESS_DISPATCH(c->dim, c->np, L_);
#undef L_
    TBDG_HIP(hipGetLastError());
    return (int)G;
}

void launch_guess_feat(const tbdg_ctx* c, const double* cells, const double* partial, int G,
                       float* feat, double* sc) {
    hipLaunchKernelGGL(k_guess_feat, dim3(nb256(c->Nc)), dim3(256), 0, c->stream, (int)c->Nc, cells,
                       partial, G, feat, sc);
    TBDG_HIP(hipGetLastError());
}

void launch_guess_inject(const tbdg_ctx* c, const double* p, const double* d1, const double* d2,
                         const double* d3, const float* y, double* out) {
    if (c->mapped)
        throw Error(TBDG_EUNSUPPORTED, "the learned guess is built for affine cells only");
    const int64_t g = nb256(c->Np);
    const unsigned G = (unsigned)(g < 2048 ? g : 2048);
#define L_(D, NP)                                                                          \
    hipLaunchKernelGGL((k_guess_inject<ipw(NP, D)>), dim3(G), dim3(256), 0, c->stream,        \
                       (int)c->Nc, p, d1, d2, d3, y, out);
    TBDG_GUESS_DISPATCH(c->dim, c->np, L_);
#undef L_
    TBDG_HIP(hipGetLastError());
}

void launch_guess_target(const tbdg_ctx* c, const double* pn, const double* p, const double* d1,
                         const double* d2, const double* d3, double* rows, double* partial,
                         float* out) {
    if (c->mapped)
        throw Error(TBDG_EUNSUPPORTED, "the learned guess is built for affine cells only");
    unsigned G = 0;
#define L_(D, NP)                                                                          \
    G = (unsigned)((c->Nc + CellBlock<D, NP>::CPB - 1) / CellBlock<D, NP>::CPB);           \
    hipLaunchKernelGGL((k_guess_gram<D, NP>), dim3(G), dim3(256), 0, c->stream, (int)c->Nc,   \
                       c->tab, pn, p, d1, d2, d3, rows, partial);
    TBDG_GUESS_DISPATCH(c->dim, c->np, L_);
#undef L_
    hipLaunchKernelGGL(k_guess_gram_scale, dim3(nb256(c->Nc)), dim3(256), 0, c->stream, (int)c->Nc,
                       rows, partial, (int)G, out);
    TBDG_HIP(hipGetLastError());
}

}  // namespace trbdg
