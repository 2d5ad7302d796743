// Cell-grid inputs and outputs of the learned pressure initial guess.
//
// Per Helmholtz solve of stage s (beta_s, right-hand side b, previous
// pressure p, the two newest increments inc1 (beta1) and inc2 (beta2)):
//   f0_K  = mean_K(inc1) / (beta1 dt),  f1_K = mean_K(inc2) / (beta2 dt),
//   div_K = -(beta_s dt / |K|) sum_{i in K} (b_i - alpha |K| W_i p_i),
// mean_K = sum_i W_i v_i (W_i: product of the Gauss weights of node i);
// network input (f0 / s_inc, f1 / s_inc, div / s_div) with s_inc, s_div the
// RMS over cells of f0 and div (1 where zero).  The network output y (cell
// averages of the correction to the fallback p + inc2) gives the guess
// p + inc2 + beta_s dt s_inc I(y), I the multilinear interpolation from the
// cell centres to the nodes.
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

// one thread per cell: f0, f1, div into cells[3][Nc]; per-block partial sums
// of f0^2 and div^2
template <int DIM, int NP>
__global__ __launch_bounds__(256) void k_guess_cells(int Nc, Tables t, const double* __restrict__ inc1,
                                                      const double* __restrict__ inc2,
                                                      const double* __restrict__ b,
                                                      const double* __restrict__ p, double c0, double c1,
                                                      double cdiv, double inv_vol, double alpha,
                                                      double* __restrict__ cells, double* partial) {
    constexpr int NB = ipw(NP, DIM);
    const int c = blockIdx.x * 256 + threadIdx.x;
    double f0 = 0.0, f1 = 0.0, dv = 0.0;
    if (c < Nc) {
        for (int i = 0; i < NB; ++i) {
            const double w = node_weight<DIM, NP>(t.Wp, i);
            const size_t gi = (size_t)c * NB + i;
            f0 += w * inc1[gi];
            f1 += w * inc2[gi];
            dv += b[gi] * inv_vol - alpha * w * p[gi];
        }
        f0 *= c0;
        f1 *= c1;
        dv *= cdiv;
        cells[c] = f0;
        cells[Nc + c] = f1;
        cells[2 * Nc + c] = dv;
    }
    const double s0 = red::block_sum(f0 * f0);
    const double s2 = red::block_sum(dv * dv);
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = s0;
        partial[gridDim.x + blockIdx.x] = s2;
    }
}

// scales from the partials (every block sums them in the same order) and the
// FP32 network input [3][Nc]; block 0 stores (s_inc, s_div) in sc
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
        feat[c] = (float)(cells[c] * ri);
        feat[Nc + c] = (float)(cells[Nc + c] * ri);
        feat[2 * Nc + c] = (float)(cells[2 * Nc + c] * rd);
    }
}

// out_i = p_i + inc2_i + beta_s dt s_inc I(y)_i, I the multilinear
// interpolation of the cell values from the cell centres (periodic)
template <int DIM, int NP>
__global__ __launch_bounds__(256) void k_guess_inject(int Nc, Geom g, Tables t,
                                                       const double* __restrict__ p,
                                                       const double* __restrict__ inc2,
                                                       const float* __restrict__ y, double bdt,
                                                       const double* __restrict__ sc,
                                                       double* __restrict__ out) {
    constexpr int NB = ipw(NP, DIM);
    const int64_t n = (int64_t)Nc * NB;
    const double f = bdt * sc[0];
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const int c = (int)(i / NB);
        int node = (int)(i % NB), rest = c;
        int lo[3] = {0, 0, 0};
        double w[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const int ca = rest % g.nc[a];
            rest /= g.nc[a];
            const double X = ca + t.xp[node % NP] - 0.5;     // position in cell-centre units
            node /= NP;
            const int i0 = (int)floor(X);
            lo[a] = i0;
            w[a] = X - i0;
        }
        double v = 0.0;
#pragma unroll
        for (int corner = 0; corner < (1 << DIM); ++corner) {
            double wt = 1.0;
            int idx = 0, stride = 1;
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                const int bit = (corner >> a) & 1;
                wt *= bit ? w[a] : 1.0 - w[a];
                int ia = lo[a] + bit;
                ia = ia < 0 ? ia + g.nc[a] : (ia >= g.nc[a] ? ia - g.nc[a] : ia);
                idx += ia * stride;
                stride *= g.nc[a];
            }
            v += wt * (double)y[idx];
        }
        out[i] = p[i] + inc2[i] + f * v;
    }
}

// out_K = mean_K(p_new - p - inc2) / (beta_s dt) / s_inc
template <int DIM, int NP>
__global__ __launch_bounds__(256) void k_guess_target(int Nc, Tables t, const double* __restrict__ pn,
                                                       const double* __restrict__ p,
                                                       const double* __restrict__ inc2, double inv_bdt,
                                                       const double* __restrict__ sc,
                                                       float* __restrict__ out) {
    constexpr int NB = ipw(NP, DIM);
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= Nc) return;
    double s = 0.0;
    for (int i = 0; i < NB; ++i) {
        const size_t gi = (size_t)c * NB + i;
        s += node_weight<DIM, NP>(t.Wp, i) * (pn[gi] - p[gi] - inc2[gi]);
    }
    out[c] = (float)(s * inv_bdt / sc[0]);
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

int launch_guess_cells(const tbdg_ctx* c, const double* inc1, const double* inc2, const double* b,
                       const double* p, double c0, double c1, double cdiv, double alpha,
                       double* cells, double* partial) {
    if (c->mapped)
        throw Error(TBDG_EUNSUPPORTED, "the learned guess is built for affine cells only");
    const unsigned G = nb256(c->Nc);
#define L_(D, NP)                                                                          \
    hipLaunchKernelGGL((k_guess_cells<D, NP>), dim3(G), dim3(256), 0, c->stream, (int)c->Nc,  \
                       c->tab, inc1, inc2, b, p, c0, c1, cdiv, 1.0 / c->geom.vol, alpha,   \
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

void launch_guess_inject(const tbdg_ctx* c, const double* p, const double* inc2, const float* y,
                         double bdt, const double* sc, double* out) {
    if (c->mapped)
        throw Error(TBDG_EUNSUPPORTED, "the learned guess is built for affine cells only");
    const int64_t g = nb256(c->Np);
    const unsigned G = (unsigned)(g < 2048 ? g : 2048);
#define L_(D, NP)                                                                          \
    hipLaunchKernelGGL((k_guess_inject<D, NP>), dim3(G), dim3(256), 0, c->stream, (int)c->Nc,  \
                       c->geom, c->tab, p, inc2, y, bdt, sc, out);
    TBDG_GUESS_DISPATCH(c->dim, c->np, L_);
#undef L_
    TBDG_HIP(hipGetLastError());
}

void launch_guess_target(const tbdg_ctx* c, const double* pn, const double* p, const double* inc2,
                         double inv_bdt, const double* sc, float* out) {
    if (c->mapped)
        throw Error(TBDG_EUNSUPPORTED, "the learned guess is built for affine cells only");
#define L_(D, NP)                                                                          \
    hipLaunchKernelGGL((k_guess_target<D, NP>), dim3(nb256(c->Nc)), dim3(256), 0, c->stream,   \
                       (int)c->Nc, c->tab, pn, p, inc2, inv_bdt, sc, out);
    TBDG_GUESS_DISPATCH(c->dim, c->np, L_);
#undef L_
    TBDG_HIP(hipGetLastError());
}

}  // namespace trbdg
