// Vector kernels and deterministic reductions for the Krylov solvers.
//
// Reductions are two-pass: a fixed grid of work-groups writes one partial sum
// each (wave64 shuffles, then LDS across the four waves), and a single
// work-group adds the partials in a fixed order.  The grid size does not
// depend on timing, so results are bitwise reproducible run to run.
#include "internal.hpp"
#include "krylov.hpp"
#include "reduce.hpp"

namespace trbdg {
namespace {

constexpr int BS = 256;

inline unsigned grid_for(int64_t n) {
    int64_t g = (n + BS - 1) / BS;
    if (g < 1) g = 1;
    if (g > 65535) g = 65535;
    return (unsigned)g;
}

using red::block_sum;

__global__ __launch_bounds__(BS) void k_axpby(int64_t n, double a, const double* x, double b,
                                              const double* y, double* out) {
    for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS)
        out[i] = a * x[i] + (y ? b * y[i] : 0.0);
}

__global__ __launch_bounds__(BS) void k_div(int64_t n, const double* x, const double* d,
                                            double* out) {
    for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS)
        out[i] = x[i] / d[i];
}

__device__ inline int64_t diag_index(int64_t i, int dim, int64_t nb) {
    return (i / (dim * nb)) * nb + (i % nb);
}

__global__ __launch_bounds__(BS) void k_div_diag_u(int64_t n, int dim, int64_t nb,
                                                   const double* x, const double* d,
                                                   double* out) {
    for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS)
        out[i] = x[i] / d[diag_index(i, dim, nb)];
}

__global__ __launch_bounds__(BS) void k_add_div_diag_u(int64_t n, int dim, int64_t nb,
                                                       const double* gz, const double* d,
                                                       double* x) {
    for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS)
        x[i] += gz[i] / d[diag_index(i, dim, nb)];
}

// partial[j * G + b] = sum over block b's slice of V_j . w
__global__ __launch_bounds__(BS) void k_dot_many(int64_t n, const double* V, int64_t ldv,
                                                 const double* w, double* partial) {
    const int j = blockIdx.y;
    const double* v = V + (int64_t)j * ldv;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS)
        acc += v[i] * w[i];
    acc = block_sum(acc);
    if (threadIdx.x == 0) partial[(int64_t)j * gridDim.x + blockIdx.x] = acc;
}

// this thread's share of sum_b p[b] (b = tid, tid + BS, ...): eight
// independent sums keep eight loads in flight (an operator kernel leaves one
// partial per block, 65 536 at 64^3 Q3), combined in a fixed order
__device__ inline double thread_sum(const double* p, int G) {
    double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int b = threadIdx.x;
    for (; b + 7 * BS < G; b += 8 * BS) {
#pragma unroll
        for (int q = 0; q < 8; ++q) a[q] += p[b + q * BS];
    }
    for (int q = 0; b < G; b += BS, ++q) a[q & 7] += p[b];
    return ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
}

// out[j] = sum_b partial[j * G + b]
__global__ __launch_bounds__(BS) void k_finish(const double* partial, int G, double* out) {
    const int j = blockIdx.x;
    double acc = thread_sum(partial + (int64_t)j * G, G);
    acc = block_sum(acc);
    if (threadIdx.x == 0) out[j] = acc;
}

__global__ __launch_bounds__(BS) void k_sub_combo(int64_t n, int k, const double* V, int64_t ldv,
                                                  const double* h, double* w) {
    for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS) {
        double s = 0.0;
        for (int j = 0; j < k; ++j) s += h[j] * V[(int64_t)j * ldv + i];
        w[i] -= s;
    }
}

// x += sum_j y_j V_j, with y_j scaled by gsc[j] when gsc is set
__global__ __launch_bounds__(BS) void k_add_combo(int64_t n, int k, const double* V, int64_t ldv,
                                                  const double* y, const double* gsc, double* x) {
    for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS) {
        double s = 0.0;
        for (int j = 0; j < k; ++j) s += (gsc ? y[j] * gsc[j] : y[j]) * V[(int64_t)j * ldv + i];
        x[i] += s;
    }
}

// ---- CG -------------------------------------------------------------------
// sc: [0] rz, [1] pAp, [2] rr, [3] rz_new, [4] alpha, [5] beta, [6] breakdown
__global__ void k_cg_alpha_finish(const double* partial, int G, double* sc) {
    double acc = 0.0;
    for (int b = threadIdx.x; b < G; b += BS) acc += partial[b];
    acc = block_sum(acc);
    if (threadIdx.x == 0) {
        sc[1] = acc;
        if (!(acc > 0.0)) {
            sc[6] = 1.0;
            sc[4] = 0.0;
        } else {
            sc[4] = sc[0] / acc;
        }
    }
}

__global__ __launch_bounds__(BS) void k_cg_update(int64_t n, const double* diag, double* x,
                                                  double* r, const double* p, const double* q,
                                                  const double* sc, double* partial) {
    const double alpha = sc[4];
    double rz = 0.0, rr = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS) {
        x[i] += alpha * p[i];
        const double ri = r[i] - alpha * q[i];
        r[i] = ri;
        rz += ri * ri / diag[i];
        rr += ri * ri;
    }
    rz = block_sum(rz);
    rr = block_sum(rr);
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = rz;
        partial[gridDim.x + blockIdx.x] = rr;
    }
}

__global__ void k_cg_beta_finish(const double* partial, int G, double* sc, int first) {
    double rz = 0.0, rr = 0.0;
    for (int b = threadIdx.x; b < G; b += BS) {
        rz += partial[b];
        rr += partial[G + b];
    }
    rz = block_sum(rz);
    rr = block_sum(rr);
    if (threadIdx.x == 0) {
        sc[2] = rr;
        sc[3] = rz;
        sc[5] = first ? 0.0 : rz / sc[0];
        sc[0] = rz;
        if (first) sc[6] = 0.0;   // clear the breakdown flag of a previous solve
    }
}

__global__ __launch_bounds__(BS) void k_cg_direction(int64_t n, const double* diag,
                                                     const double* r, double* p,
                                                     const double* sc) {
    const double beta = sc[5];
    for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS)
        p[i] = r[i] / diag[i] + beta * p[i];
}

__global__ __launch_bounds__(BS) void k_cg_init_partials(int64_t n, const double* diag,
                                                         const double* r, double* p,
                                                         double* partial) {
    double rz = 0.0, rr = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS) {
        const double ri = r[i];
        const double zi = ri / diag[i];
        p[i] = zi;
        rz += ri * zi;
        rr += ri * ri;
    }
    rz = block_sum(rz);
    rr = block_sum(rr);
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = rz;
        partial[gridDim.x + blockIdx.x] = rr;
    }
}


__global__ __launch_bounds__(BS) void k_recip(int64_t n, const double* d, double* out) {
    for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS)
        out[i] = 1.0 / d[i];
}

// CG direction: p = r * invd + beta p   (beta = sc[5], 0 on the first iteration)
__global__ __launch_bounds__(BS) void k_cg_dir(int64_t n, const double* invd, const double* r,
                                               double* p, const double* sc) {
    const double beta = sc[5];
    for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS)
        p[i] = r[i] * invd[i] + beta * p[i];
}

// CG update: every block first adds the Ga partial sums p.q of the operator
// kernel (same order in every block) and forms alpha = sc[slot] / p.q;
// then x += alpha p, r -= alpha q and one partial (r.(invd r), r.r) per
// block.  Block 0 records alpha (sc[4]), p.q (sc[1]) and a breakdown flag.
__global__ __launch_bounds__(BS) void k_cg_upd(int64_t n, const double* invd, double* x, double* r,
                                               const double* p, const double* q, double* sc,
                                               const double* pa, int Ga, int slot,
                                               double* partial) {
    __shared__ double s_alpha;
    double pq = 0.0;
    for (int b = threadIdx.x; b < Ga; b += BS) pq += pa[b];
    pq = block_sum(pq);
    if (threadIdx.x == 0) {
        const bool ok = pq > 0.0;
        s_alpha = ok ? sc[slot] / pq : 0.0;
        if (blockIdx.x == 0) {
            sc[1] = pq;
            sc[4] = s_alpha;
            if (!ok) sc[6] = 1.0;
        }
    }
    __syncthreads();
    const double alpha = s_alpha;
    double rz = 0.0, rr = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS) {
        x[i] += alpha * p[i];
        const double ri = r[i] - alpha * q[i];
        r[i] = ri;
        rz += ri * ri * invd[i];
        rr += ri * ri;
    }
    rz = block_sum(rz);
    rr = block_sum(rr);
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = rz;
        partial[gridDim.x + blockIdx.x] = rr;
    }
}

// first CG direction: p = invd r, partial rz and rr
__global__ __launch_bounds__(BS) void k_cg_start(int64_t n, const double* invd, const double* r,
                                                 double* p, double* partial) {
    double rz = 0.0, rr = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS) {
        const double ri = r[i];
        const double zi = ri * invd[i];
        p[i] = zi;
        rz += ri * zi;
        rr += ri * ri;
    }
    rz = block_sum(rz);
    rr = block_sum(rr);
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = rz;
        partial[gridDim.x + blockIdx.x] = rr;
    }
}

// GMRES multi-dot: partial[j*G + b] = V_j . w over block b's slice for the
// 8 vectors of group blockIdx.y; group 0 also sums w.w into slot k.
__global__ __launch_bounds__(BS) void k_mdot8(int64_t n, int k, const double* V, int64_t ldv,
                                              const double* w, double* partial) {
    const int j0 = blockIdx.y * 8;
    const int jn = min(8, k - j0);
    const int G = gridDim.x;
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    double ww = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < n; i += (int64_t)G * BS) {
        const double wi = w[i];
        if (blockIdx.y == 0) ww += wi * wi;
#pragma unroll
        for (int jj = 0; jj < 8; ++jj)
            if (jj < jn) acc[jj] += V[(int64_t)(j0 + jj) * ldv + i] * wi;
    }
    for (int jj = 0; jj < 8; ++jj) {
        const double s = block_sum(acc[jj]);
        if (threadIdx.x == 0 && jj < jn) partial[(size_t)(j0 + jj) * G + blockIdx.x] = s;
    }
    if (blockIdx.y == 0) {
        const double s = block_sum(ww);
        if (threadIdx.x == 0) partial[(size_t)k * G + blockIdx.x] = s;
    }
}

// GMRES update with fused norm partials: w -= sum_j h_j gsc_j V_j (the V_j
// unnormalised, gsc_j their inverse norms), partial |w|^2
__global__ __launch_bounds__(BS) void k_update_norm(int64_t n, int k, const double* V, int64_t ldv,
                                                    const double* h, const double* gsc, double* w,
                                                    double* partial) {
    __shared__ double s_cf[64];
    for (int j = threadIdx.x; j < k; j += BS) s_cf[j] = gsc ? h[j] * gsc[j] : h[j];
    __syncthreads();
    double nn = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS) {
        double s = w[i];
        for (int j = 0; j < k; ++j) s -= s_cf[j] * V[(int64_t)j * ldv + i];
        w[i] = s;
        nn += s * s;
    }
    nn = block_sum(nn);
    if (threadIdx.x == 0) partial[blockIdx.x] = nn;
}

// GMRES restart without an operator apply: x += D^{-1} sum_{j<k} y_j gsc_j V_j
// and V_0 = sum_{j<=k} cr_j gsc_j V_j (the residual of the updated x in the
// Krylov basis), with the partial sums of |V_0|^2.  Each thread reads V_0[i]
// before it overwrites it.
__global__ __launch_bounds__(BS) void k_gm_restart(int64_t n, int dim, int64_t nb, int k, double* V,
                                                   int64_t ldv, const double* y, const double* cr,
                                                   const double* gsc, const double* invd, double* x,
                                                   double* partial, double* xcomb) {
    __shared__ double s_y[64], s_c[64];
    for (int j = threadIdx.x; j <= k; j += BS) {
        s_y[j] = j < k ? y[j] * gsc[j] : 0.0;
        s_c[j] = cr[j] * gsc[j];
    }
    __syncthreads();
    double nn = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS) {
        double sx = 0.0, sr = 0.0;
        for (int j = 0; j <= k; ++j) {
            const double v = V[(int64_t)j * ldv + i];
            sx += s_y[j] * v;
            sr += s_c[j] * v;
        }
        if (xcomb) xcomb[i] = sx;
        else x[i] += sx * invd[diag_index(i, dim, nb)];
        V[i] = sr;
        nn += sr * sr;
    }
    nn = block_sum(nn);
    if (threadIdx.x == 0) partial[blockIdx.x] = nn;
}

// out[j] = gsc[j] * sum_b partial[j * G + b] for j < k; out[k] = the plain
// sum of slot k (w . w)
__global__ __launch_bounds__(BS) void k_finish_gs(const double* partial, int G, int k,
                                                  const double* gsc, double* out, double* hout) {
    const int j = blockIdx.x;
    double acc = thread_sum(partial + (int64_t)j * G, G);
    acc = block_sum(acc);
    if (threadIdx.x == 0) {
        const double v = j < k && gsc ? gsc[j] * acc : acc;
        out[j] = v;
        if (hout) {
            hout[j] = v;
            __threadfence_system();
        }
    }
}

// nn = sum of the partials; inv = 1 / sqrt(nn) (1 when nn is not positive)
__global__ __launch_bounds__(BS) void k_finish_inv_norm(const double* partial, int G, double* nn,
                                                        double* inv, double* hnn) {
    double acc = 0.0;
    for (int b = threadIdx.x; b < G; b += BS) acc += partial[b];
    acc = block_sum(acc);
    if (threadIdx.x == 0) {
        if (nn) nn[0] = acc;
        inv[0] = acc > 0.0 ? 1.0 / sqrt(acc) : 1.0;
        if (hnn) {
            hnn[0] = acc;
            __threadfence_system();
        }
    }
}

}  // namespace

// address in host_out (as seen by the device) of a scalar slot of red_out
double* host_mirror(const tbdg_ctx* c, const double* dev) {
    if (!c->host_dev || dev < c->red_out || dev >= c->red_out + 128)
        throw Error(TBDG_EINVAL, "scalar slot outside the mirrored range");
    return c->host_dev + (dev - c->red_out);
}

int reduce_grid(int64_t n, int cap) {
    int64_t g = (n + BS - 1) / BS;
    if (g > cap) g = cap;
    if (g < 1) g = 1;
    return (int)g;
}

void vec_axpby(hipStream_t s, int64_t n, double a, const double* x, double b, const double* y,
               double* out) {
    hipLaunchKernelGGL(k_axpby, dim3(grid_for(n)), dim3(BS), 0, s, n, a, x, b, y, out);
    TBDG_HIP(hipGetLastError());
}

void vec_scale_copy(hipStream_t s, int64_t n, double a, const double* x, double* out) {
    vec_axpby(s, n, a, x, 0.0, nullptr, out);
}

void vec_div(hipStream_t s, int64_t n, const double* x, const double* d, double* out) {
    hipLaunchKernelGGL(k_div, dim3(grid_for(n)), dim3(BS), 0, s, n, x, d, out);
    TBDG_HIP(hipGetLastError());
}

void vec_div_diag_u(hipStream_t s, int64_t n, int dim, int64_t nb, const double* x,
                    const double* d, double* out) {
    hipLaunchKernelGGL(k_div_diag_u, dim3(grid_for(n)), dim3(BS), 0, s, n, dim, nb, x, d, out);
    TBDG_HIP(hipGetLastError());
}

void vec_add_div_diag_u(hipStream_t s, int64_t n, int dim, int64_t nb, const double* gz,
                        const double* d, double* x) {
    hipLaunchKernelGGL(k_add_div_diag_u, dim3(grid_for(n)), dim3(BS), 0, s, n, dim, nb, gz, d, x);
    TBDG_HIP(hipGetLastError());
}

void dot_many(tbdg_ctx* c, int64_t n, int k, const double* V, int64_t ldv, const double* w,
              double* dev_out) {
    const int G = reduce_grid(n, c->red_blocks / (k > 0 ? k : 1) < 1024 ? c->red_blocks / (k > 0 ? k : 1) : 1024);
    hipLaunchKernelGGL(k_dot_many, dim3(G, k), dim3(BS), 0, c->stream, n, V, ldv, w, c->red_part);
    hipLaunchKernelGGL(k_finish, dim3(k), dim3(BS), 0, c->stream, c->red_part, G, dev_out);
    TBDG_HIP(hipGetLastError());
}

void dot2(tbdg_ctx* c, int64_t n, const double* a, const double* b, double* dev_out) {
    dot_many(c, n, 1, a, 0, b, dev_out);
}

void vec_sub_combo(hipStream_t s, int64_t n, int k, const double* V, int64_t ldv,
                   const double* h, double* w) {
    hipLaunchKernelGGL(k_sub_combo, dim3(grid_for(n)), dim3(BS), 0, s, n, k, V, ldv, h, w);
    TBDG_HIP(hipGetLastError());
}

void vec_add_combo(hipStream_t s, int64_t n, int k, const double* V, int64_t ldv,
                   const double* y, const double* gsc, double* x) {
    hipLaunchKernelGGL(k_add_combo, dim3(grid_for(n)), dim3(BS), 0, s, n, k, V, ldv, y, gsc, x);
    TBDG_HIP(hipGetLastError());
}

void vec_recip(hipStream_t s, int64_t n, const double* d, double* out) {
    hipLaunchKernelGGL(k_recip, dim3(grid_for(n)), dim3(BS), 0, s, n, d, out);
    TBDG_HIP(hipGetLastError());
}

void cg_start(tbdg_ctx* c, int64_t n, const double* invd, const double* r, double* p, double* sc,
              double* up, int Gu) {
    hipLaunchKernelGGL(k_cg_start, dim3(Gu), dim3(BS), 0, c->stream, n, invd, r, p, up);
    hipLaunchKernelGGL(k_cg_beta_finish, dim3(1), dim3(BS), 0, c->stream, up, Gu, sc, 1);
    TBDG_HIP(hipGetLastError());
}

void cg_alpha_finish(const tbdg_ctx* c, int G, const double* partial, double* sc) {
    hipLaunchKernelGGL(k_cg_alpha_finish, dim3(1), dim3(BS), 0, c->stream, partial, G, sc);
    TBDG_HIP(hipGetLastError());
}

void cg_dir(tbdg_ctx* c, int64_t n, const double* invd, const double* r, double* p, const double* sc) {
    hipLaunchKernelGGL(k_cg_dir, dim3(grid_for(n)), dim3(BS), 0, c->stream, n, invd, r, p, sc);
    TBDG_HIP(hipGetLastError());
}

void cg_upd(tbdg_ctx* c, int64_t n, const double* invd, double* x, double* r, const double* p,
            const double* q, double* sc, const double* pa, int Ga, int slot, double* up, int Gu) {
    hipLaunchKernelGGL(k_cg_upd, dim3(Gu), dim3(BS), 0, c->stream, n, invd, x, r, p, q, sc, pa,
                       Ga, slot, up);
    TBDG_HIP(hipGetLastError());
}

void gm_dots(tbdg_ctx* c, int64_t n, int k, const double* V, int64_t ldv, const double* w,
             const double* gsc, double* dev_out) {
    const int groups = (k + 7) / 8;
    // blocks per group of 8 vectors: enough to fill the chip with all groups
    // together, few enough that each thread streams a dozen or more entries
    // before its eight block reductions ((k + 1) * G <= 62 * 4096 slots)
    const int G = reduce_grid(n, groups >= 2 ? 1024 : 2048);
    hipLaunchKernelGGL(k_mdot8, dim3(G, groups), dim3(BS), 0, c->stream, n, k, V, ldv, w,
                       c->red_part);
    hipLaunchKernelGGL(k_finish_gs, dim3(k + 1), dim3(BS), 0, c->stream, c->red_part, G, k, gsc,
                       dev_out, host_mirror(c, dev_out));
    TBDG_HIP(hipGetLastError());
}

void gm_finish_dots(tbdg_ctx* c, int G, int k, const double* part, const double* gsc,
                    double* dev_out) {
    hipLaunchKernelGGL(k_finish_gs, dim3(k + 1), dim3(BS), 0, c->stream, part, G, k, gsc, dev_out,
                       host_mirror(c, dev_out));
    TBDG_HIP(hipGetLastError());
}

void gm_update_norm(tbdg_ctx* c, int64_t n, int k, const double* V, int64_t ldv, const double* h,
                    const double* gsc, double* w, double* dev_nn, double* gsc_next) {
    const int G = reduce_grid(n, 4096);
    double* part = c->red_part + 62 * 4096;
    hipLaunchKernelGGL(k_update_norm, dim3(G), dim3(BS), 0, c->stream, n, k, V, ldv, h, gsc, w,
                       part);
    hipLaunchKernelGGL(k_finish_inv_norm, dim3(1), dim3(BS), 0, c->stream, part, G, dev_nn,
                       gsc_next, host_mirror(c, dev_nn));
    TBDG_HIP(hipGetLastError());
}

void gm_restart(tbdg_ctx* c, int64_t n, int k, double* V, int64_t ldv, const double* y,
                const double* cr, const double* gsc, const double* invd, double* x, double* dev_nn,
                double* gsc0, double* xcomb) {
    const int G = reduce_grid(n, 4096);
    double* part = c->red_part + 62 * 4096;
    hipLaunchKernelGGL(k_gm_restart, dim3(G), dim3(BS), 0, c->stream, n, c->dim, c->nbu, k, V, ldv,
                       y, cr, gsc, invd, x, part, xcomb);
    hipLaunchKernelGGL(k_finish_inv_norm, dim3(1), dim3(BS), 0, c->stream, part, G, dev_nn, gsc0,
                       host_mirror(c, dev_nn));
    TBDG_HIP(hipGetLastError());
}

void kr_dots(hipStream_t st, int64_t n, int k, const double* V, int64_t ldv, const double* w,
             double* part, int G, double* out) {
    hipLaunchKernelGGL(k_mdot8, dim3(G, (k + 7) / 8), dim3(BS), 0, st, n, k, V, ldv, w, part);
    hipLaunchKernelGGL(k_finish_gs, dim3(k + 1), dim3(BS), 0, st, part, G, k, nullptr, out, nullptr);
    TBDG_HIP(hipGetLastError());
}

void kr_update_norm(hipStream_t st, int64_t n, int k, const double* V, int64_t ldv, const double* h,
                    double* w, double* part, int G, double* nn, double* inv) {
    hipLaunchKernelGGL(k_update_norm, dim3(G), dim3(BS), 0, st, n, k, V, ldv, h, nullptr, w, part);
    hipLaunchKernelGGL(k_finish_inv_norm, dim3(1), dim3(BS), 0, st, part, G, nn, inv, nullptr);
    TBDG_HIP(hipGetLastError());
}

void gm_norm_inv(tbdg_ctx* c, int64_t n, const double* v, double* dev_nn, double* inv) {
    const int G = reduce_grid(n, 1024);
    hipLaunchKernelGGL(k_dot_many, dim3(G, 1), dim3(BS), 0, c->stream, n, v, (int64_t)0, v,
                       c->red_part);
    hipLaunchKernelGGL(k_finish_inv_norm, dim3(1), dim3(BS), 0, c->stream, c->red_part, G, dev_nn,
                       inv, host_mirror(c, dev_nn));
    TBDG_HIP(hipGetLastError());
}

void cg_alpha(tbdg_ctx* c, int64_t n, const double* p, const double* q, double* sc) {
    const int G = reduce_grid(n, 1024);
    hipLaunchKernelGGL(k_dot_many, dim3(G, 1), dim3(BS), 0, c->stream, n, p, 0, q, c->red_part);
    hipLaunchKernelGGL(k_cg_alpha_finish, dim3(1), dim3(BS), 0, c->stream, c->red_part, G, sc);
    TBDG_HIP(hipGetLastError());
}

void cg_update(tbdg_ctx* c, int64_t n, const double* diag, double* x, double* r, const double* p,
               const double* q, double* sc) {
    const int G = reduce_grid(n, 4096);
    hipLaunchKernelGGL(k_cg_update, dim3(G), dim3(BS), 0, c->stream, n, diag, x, r, p, q, sc,
                       c->red_part);
    hipLaunchKernelGGL(k_cg_beta_finish, dim3(1), dim3(BS), 0, c->stream, c->red_part, G, sc, 0);
    TBDG_HIP(hipGetLastError());
}

void cg_direction(hipStream_t s, int64_t n, const double* diag, const double* r, double* p,
                  const double* sc) {
    hipLaunchKernelGGL(k_cg_direction, dim3(grid_for(n)), dim3(BS), 0, s, n, diag, r, p, sc);
    TBDG_HIP(hipGetLastError());
}

void cg_init(tbdg_ctx* c, int64_t n, const double* diag, const double* r, double* p, double* sc) {
    const int G = reduce_grid(n, 1024);
    hipLaunchKernelGGL(k_cg_init_partials, dim3(G), dim3(BS), 0, c->stream, n, diag, r, p,
                       c->red_part);
    hipLaunchKernelGGL(k_cg_beta_finish, dim3(1), dim3(BS), 0, c->stream, c->red_part, G, sc, 1);
    TBDG_HIP(hipGetLastError());
}

}  // namespace trbdg
