// Multigrid kernels for Helmholtz operators H = alpha M + K (the pressure's,
// and one velocity component's with Dirichlet walls): the FP32 (or
// BF16-storage / FP32-arithmetic) level operator fused with one step of the
// Chebyshev smoother, the nested-space transfers, the FP64 coarse solve and
// the FP64 glue of flexible CG and of the velocity preconditioner.
//
// Smoother (Chebyshev acceleration of the Jacobi-preconditioned system on
// [lo, hi], theta = (hi + lo)/2): d_0 = D^{-1} r_0 / theta, then per step
//   x_k = x_{k-1} + d_{k-1},  r_k = r_{k-1} - H d_{k-1},
//   d_k = c1_k d_{k-1} + c2_k D^{-1} r_k.
// Each step is one launch of k_level; the operand d_{k-1} is the only vector
// read at neighbour cells, so d is ping-ponged and x, r are updated in place.
#include <hip/hip_runtime.h>

#include "internal.hpp"
#include "lines.hpp"
#include "reduce.hpp"

namespace trbdg {
namespace {

using namespace lines;

// ---- storage types ------------------------------------------------------------
// float, or bfloat16 (upper half of an IEEE binary32; round to nearest even on
// store, quiet NaN kept) with float arithmetic.
template <typename S>
struct Sto;
template <>
struct Sto<float> {
    __device__ static inline float ld(const float* p, size_t i) { return p[i]; }
    __device__ static inline float put(float* p, size_t i, float v) {
        p[i] = v;
        return v;
    }
};
template <>
struct Sto<uint16_t> {
    __device__ static inline float ld(const uint16_t* p, size_t i) {
        return __uint_as_float((unsigned)p[i] << 16);
    }
    __device__ static inline uint16_t round(float v) {
        const unsigned u = __float_as_uint(v);
        if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
        return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
    }
    // stores the rounded value and returns it as float
    __device__ static inline float put(uint16_t* p, size_t i, float v) {
        const uint16_t h = round(v);
        p[i] = h;
        return __uint_as_float((unsigned)h << 16);
    }
};

// One smoother step on one level (modes above):
//   MG_PRE1  x = d;      r = b - H d;  d' = c1 d + c2 D^{-1} r
//   MG_STEP  x += d;     r -= H d;     d' = c1 d + c2 D^{-1} r
//   MG_LAST  x += d;     r -= H d
//   MG_RES   r = b - H x;              d' = c2 D^{-1} r
//   MG_ZFIN  as MG_STEP, but writes only z = x + d' in FP64 and per-block
//           partial sums z.r64 and z.q64 (the last step of the finest level;
//           z, r64, q64 hold zs values per cell, r64 / q64 / partial may be
//           null)
// The operator is the same line-structured SIP form as the FP64 kernel:
// neighbour traces (value, normal derivative) gathered in LDS, one work item
// per (cell, direction, grid line), then mass term and directions summed.
template <int DIM, int NP, typename S, int MODE>
__global__ __launch_bounds__(256) void k_level(Geom g, LineGeom lg, LevelTabF t, float cm,
                                                float c1, float c2, const S* __restrict__ dop,
                                                S* __restrict__ x, S* __restrict__ r,
                                                const S* __restrict__ b,
                                                const float* __restrict__ invd,
                                                S* __restrict__ dout, int Nc,
                                                double* __restrict__ z,
                                                const double* __restrict__ r64,
                                                const double* __restrict__ q64,
                                                double* __restrict__ partial, int zs) {
    using L = Lay<DIM, NP>;
    using F = FaceLay<DIM, NP>;
    using T = Sto<S>;
    constexpr int NB = F::NB, NF = F::NF, CPB = F::CPB;
    constexpr int NFACE = 2 * DIM * NF;
    __shared__ float s_p[256];
    __shared__ float s_y[DIM][256];
    __shared__ float s_f[CPB * NFACE * 2];
    __shared__ int s_nbr[CPB * 2 * DIM];
    const S* op = MODE == MG_RES ? x : dop;
    const int tid = threadIdx.x;
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    const int lc = tid / NB, nd = tid % NB;
    const int cell = blk * CPB + lc;
    const bool active = lc < CPB && cell < Nc;
    const size_t gi = (size_t)cell * NB + nd;
    const float pown = active ? T::ld(op, gi) : 0.0f;
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
    for (int it = nd; lc < CPB && it < NFACE; it += NB) {
        const int face = it / NF, tt = it % NF;
        const int a = face >> 1, s = face & 1;
        float v = 0.0f, d = 0.0f;
        const int nbr = s_nbr[lc * 2 * DIM + face];
        if (nbr >= 0) {
#pragma unroll
            for (int m = 0; m < NP; ++m) {
                const float pv = T::ld(op, (size_t)nbr * NB + L::node(a, m, tt));
                v += (s ? t.L0[m] : t.L1[m]) * pv;
                d += (s ? t.dL0[m] : t.dL1[m]) * pv;
            }
        }
        s_f[2 * (lc * NFACE + it)] = v;
        s_f[2 * (lc * NFACE + it) + 1] = d;
    }
    __syncthreads();
    constexpr int ITEMS = CPB * DIM * NF;
    for (int it = tid; it < ITEMS; it += 256) {
        const int lc2 = it / (DIM * NF);
        const int a = (it % (DIM * NF)) / NF, ln = it % NF;
        if (blk * CPB + lc2 >= Nc) continue;
        const int base = lc2 * NB;
        float pp[NP];
        float p0 = 0.0f, p1 = 0.0f;
#pragma unroll
        for (int m = 0; m < NP; ++m) {
            pp[m] = s_p[base + L::node(a, m, ln)];
            p0 += t.L0[m] * pp[m];
            p1 += t.L1[m] * pp[m];
        }
        const bool hl = s_nbr[lc2 * 2 * DIM + 2 * a] >= 0;
        const bool hr = s_nbr[lc2 * 2 * DIM + 2 * a + 1] >= 0;
        float X0, Y0, X1, Y1;
        if (hl) {
            const int rl = 2 * (lc2 * NFACE + (2 * a) * NF + ln);
            X0 = 0.5f * s_f[rl + 1] - t.Cr * s_f[rl];
            Y0 = 0.5f * s_f[rl];
        } else {
            // no neighbour: traces of the own cell's mirror image (LineGeom::wall)
            float q0 = 0.0f;
#pragma unroll
            for (int m = 0; m < NP; ++m) q0 += t.dL0[m] * pp[m];
            X0 = t.wall * (0.5f * q0 + t.Cr * p0);
            Y0 = -t.wall * 0.5f * p0;
        }
        if (hr) {
            const int rr = 2 * (lc2 * NFACE + (2 * a + 1) * NF + ln);
            X1 = -0.5f * s_f[rr + 1] - t.Cr * s_f[rr];
            Y1 = 0.5f * s_f[rr];
        } else {
            float q1 = 0.0f;
#pragma unroll
            for (int m = 0; m < NP; ++m) q1 += t.dL1[m] * pp[m];
            X1 = t.wall * (t.Cr * p1 - 0.5f * q1);
            Y1 = -t.wall * 0.5f * p1;
        }
        float wt = 1.0f;
        if (DIM == 2) wt = t.W[ln];
        else wt = t.W[ln % NP] * t.W[ln / NP];
        const float sd = t.sdiff[a] * wt;
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            float s = 0.0f;
#pragma unroll
            for (int j = 0; j < NP; ++j) s += t.A[i * NP + j] * pp[j];
            s += t.L0[i] * X0 - t.dL0[i] * Y0 + t.L1[i] * X1 + t.dL1[i] * Y1;
            s_y[a][base + L::node(a, i, ln)] = sd * s;
        }
    }
    __syncthreads();
    double zr = 0.0, zq = 0.0;
    if (active) {
        float wn = 1.0f;
#pragma unroll
        for (int a = 0; a < DIM; ++a) wn *= t.W[L::coord(nd, a)];
        float y = cm * wn * pown;
#pragma unroll
        for (int a = 0; a < DIM; ++a) y += s_y[a][tid];
        const float id = MODE == MG_LAST ? 0.0f : invd[gi];
        if (MODE == MG_PRE1) {
            T::put(x, gi, pown);
            const float rn = T::put(r, gi, T::ld(b, gi) - y);
            T::put(dout, gi, c1 * pown + c2 * id * rn);
        } else if (MODE == MG_STEP) {
            T::put(x, gi, T::ld(x, gi) + pown);
            const float rn = T::put(r, gi, T::ld(r, gi) - y);
            T::put(dout, gi, c1 * pown + c2 * id * rn);
        } else if (MODE == MG_LAST) {
            T::put(x, gi, T::ld(x, gi) + pown);
            T::put(r, gi, T::ld(r, gi) - y);
        } else if (MODE == MG_RES) {
            const float rn = T::put(r, gi, T::ld(b, gi) - y);
            T::put(dout, gi, c2 * id * rn);
        } else {   // MG_ZFIN
            const float xn = T::ld(x, gi) + pown;
            const float rn = T::ld(r, gi) - y;
            const float dn = c1 * pown + c2 * id * rn;
            const double zi = (double)xn + (double)dn;
            const size_t zi_idx = (size_t)cell * zs + nd;
            z[zi_idx] = zi;
            if (r64) zr = zi * r64[zi_idx];
            if (q64) zq = zi * q64[zi_idx];
        }
    }
    if (MODE == MG_ZFIN && partial) {
        zr = red::block_sum(zr);
        zq = red::block_sum(zq);
        if (tid == 0) {
            partial[blockIdx.x] = zr;
            partial[gridDim.x + blockIdx.x] = zq;
        }
    }
}

// ---- transfers ----------------------------------------------------------------
// Coarse space Q_1 (2 nodes per direction).  HT = 0: p-transfer on the same
// cell, T[0][i][j] = (Q_1 basis j)(fine node i).  HT = 1: h-transfer,
// T[b][i][j] = (parent Q_1 basis j)((b + child node i) / 2).

// b_c = P^T r_f (one thread per coarse node); if d0 is given also the first
// smoother direction of the coarse level, d0 = c2 D^{-1} b_c.
template <int DIM, int NF, typename S, int HT>
__global__ __launch_bounds__(256) void k_restrict(TransferTab tt, const S* __restrict__ rf,
                                                   float* __restrict__ bc, float* __restrict__ d0,
                                                   const float* __restrict__ invd, float c2,
                                                   int ncx, int ncy, int ncz, int Ncc) {
    constexpr int NBC = 1 << DIM;
    constexpr int NBF = ipow(NF, DIM);
    using T = Sto<S>;
    const int gid = blockIdx.x * 256 + threadIdx.x;
    if (gid >= Ncc * NBC) return;
    const int C = gid / NBC, J = gid % NBC;
    const int jx = J & 1, jy = (J >> 1) & 1, jz = (J >> 2) & 1;
    float acc = 0.0f;
    if (HT == 0) {
        for (int I = 0; I < NBF; ++I) {
            const int ix = I % NF, iy = (I / NF) % NF, iz = I / (NF * NF);
            float w = tt.T[0][ix][jx] * tt.T[0][iy][jy];
            if (DIM == 3) w *= tt.T[0][iz][jz];
            acc += w * T::ld(rf, (size_t)C * NBF + I);
        }
    } else {
        const int cx = C % ncx, cy = (C / ncx) % ncy, cz = C / (ncx * ncy);
        const int fnx = 2 * ncx, fny = 2 * ncy;
        for (int ch = 0; ch < NBC; ++ch) {
            const int bx = ch & 1, by = (ch >> 1) & 1, bz = (ch >> 2) & 1;
            const int fc = (2 * cx + bx) + fnx * ((2 * cy + by) + (DIM == 3 ? fny * (2 * cz + bz) : 0));
            for (int I = 0; I < NBF; ++I) {
                const int ix = I & 1, iy = (I >> 1) & 1, iz = (I >> 2) & 1;
                float w = tt.T[bx][ix][jx] * tt.T[by][iy][jy];
                if (DIM == 3) w *= tt.T[bz][iz][jz];
                acc += w * T::ld(rf, (size_t)fc * NBF + I);
            }
        }
    }
    bc[gid] = acc;
    if (d0) d0[gid] = c2 * invd[gid] * acc;
}

// x_f += P (x_c + d_c) (one thread per fine node); d_c may be null.
template <int DIM, int NF, typename S, int HT>
__global__ __launch_bounds__(256) void k_prolong(TransferTab tt, S* __restrict__ xf,
                                                  const float* __restrict__ xc,
                                                  const float* __restrict__ dc, int fnx, int fny,
                                                  int Ncf) {
    constexpr int NBC = 1 << DIM;
    constexpr int NBF = ipow(NF, DIM);
    using T = Sto<S>;
    const int gid = blockIdx.x * 256 + threadIdx.x;
    if (gid >= Ncf * NBF) return;
    const int c = gid / NBF, I = gid % NBF;
    int C = c, bx = 0, by = 0, bz = 0;
    if (HT == 1) {
        const int fx = c % fnx, fy = (c / fnx) % fny, fz = c / (fnx * fny);
        bx = fx & 1;
        by = fy & 1;
        bz = fz & 1;
        const int ncx = fnx / 2, ncy = fny / 2;
        C = (fx >> 1) + ncx * ((fy >> 1) + (DIM == 3 ? ncy * (fz >> 1) : 0));
    }
    const int ix = I % NF, iy = (I / NF) % NF, iz = I / (NF * NF);
    float acc = 0.0f;
#pragma unroll
    for (int J = 0; J < NBC; ++J) {
        const int jx = J & 1, jy = (J >> 1) & 1, jz = (J >> 2) & 1;
        float w = tt.T[bx][ix][jx] * tt.T[by][iy][jy];
        if (DIM == 3) w *= tt.T[bz][iz][jz];
        const size_t ci = (size_t)C * NBC + J;
        acc += w * (xc[ci] + (dc ? dc[ci] : 0.0f));
    }
    T::put(xf, gid, T::ld(xf, gid) + acc);
}

// Coarsest level: x = H^{-1} b with the FP64 inverse (one wave per row).
__global__ __launch_bounds__(256) void k_coarse(const double* __restrict__ Ainv,
                                                 const float* __restrict__ b,
                                                 float* __restrict__ x, int n) {
    const int row = blockIdx.x * 4 + threadIdx.x / 64;
    const int lane = threadIdx.x % 64;
    double acc = 0.0;
    if (row < n)
        for (int j = lane; j < n; j += 64) acc += Ainv[(size_t)row * n + j] * (double)b[j];
    acc = red::wave_sum(acc);
    if (row < n && lane == 0) x[row] = (float)acc;
}

// ---- the coarse end of a V-cycle in one workgroup --------------------------------
// Every Q1 level from fc.lv[0] down to the coarsest lives in LDS; each
// smoother step, transfer and the coarse solve is one pass of the block's
// 1024 threads over the level's nodes, separated by block barriers.  The
// per-node arithmetic is k_level's and k_restrict's / k_prolong's
// (h-transfer); the coarse solve multiplies by the same FP64 inverse.

// neighbour of a cell with coordinates ci along direction a, side s (0 left,
// 1 right), or -1 at a wall
template <int DIM>
__device__ inline int fz_nbr(const int* nc, const int* per, const int* ci, int cell, int a, int s) {
    int stride = 1;
    for (int e = 0; e < a; ++e) stride *= nc[e];
    if (s == 0) return ci[a] > 0 ? cell - stride : (per[a] ? cell + (nc[a] - 1) * stride : -1);
    return ci[a] < nc[a] - 1 ? cell + stride : (per[a] ? cell - (nc[a] - 1) * stride : -1);
}

// threads of the single-workgroup cycle: 1024 in 2D; 512 in 3D, where a
// cell's eight nodes need twice the registers
template <int DIM>
constexpr int fz_threads() { return DIM == 2 ? FUSE_THREADS : FUSE_THREADS / 2; }

// the NB = 2^DIM values of one cell of a Q1 level in LDS (16-byte loads)
template <int DIM>
__device__ inline void fz_load(const float* p, int cell, float* v) {
    constexpr int NB = 1 << DIM;
    const float4* q = reinterpret_cast<const float4*>(p + cell * NB);
#pragma unroll
    for (int k = 0; k < NB / 4; ++k) {
        const float4 t = q[k];
        v[4 * k] = t.x;
        v[4 * k + 1] = t.y;
        v[4 * k + 2] = t.z;
        v[4 * k + 3] = t.w;
    }
}

// y = (H p) at the NB nodes of one cell of a Q1 level in LDS: the per-node
// arithmetic of k_level, each line's neighbour traces formed once per cell
template <int DIM>
__device__ void fz_apply(const FusedCycle& fc, const FusedLv& L, const float* p, int cell, float* y) {
    constexpr int NB = 1 << DIM;
    int ci[3] = {0, 0, 0};
    int rr = cell;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        ci[a] = rr % L.nc[a];
        rr /= L.nc[a];
    }
    float pv[NB];
    fz_load<DIM>(p, cell, pv);
#pragma unroll
    for (int n = 0; n < NB; ++n) {
        float wn = 1.0f;
#pragma unroll
        for (int a = 0; a < DIM; ++a) wn *= fc.W[(n >> a) & 1];
        y[n] = L.cm * wn * pv[n];
    }
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const int lf = fz_nbr<DIM>(L.nc, fc.periodic, ci, cell, a, 0);
        const int rt = fz_nbr<DIM>(L.nc, fc.periodic, ci, cell, a, 1);
        float pl[NB], pr[NB];
        if (lf >= 0) fz_load<DIM>(p, lf, pl);
        if (rt >= 0) fz_load<DIM>(p, rt, pr);
#pragma unroll
        for (int n0 = 0; n0 < NB; ++n0) {
            if ((n0 >> a) & 1) continue;        // one line per node with coordinate a = 0
            const int n1 = n0 | (1 << a);
            const float pp0 = pv[n0], pp1 = pv[n1];
            const float p0 = fc.L0[0] * pp0 + fc.L0[1] * pp1;
            const float p1 = fc.L1[0] * pp0 + fc.L1[1] * pp1;
            float X0, Y0, X1, Y1;
            if (lf >= 0) {
                const float v = fc.L1[0] * pl[n0] + fc.L1[1] * pl[n1];
                const float d = fc.dL1[0] * pl[n0] + fc.dL1[1] * pl[n1];
                X0 = 0.5f * d - fc.Cr * v;
                Y0 = 0.5f * v;
            } else {
                const float q0 = fc.dL0[0] * pp0 + fc.dL0[1] * pp1;
                X0 = fc.wall * (0.5f * q0 + fc.Cr * p0);
                Y0 = -fc.wall * 0.5f * p0;
            }
            if (rt >= 0) {
                const float v = fc.L0[0] * pr[n0] + fc.L0[1] * pr[n1];
                const float d = fc.dL0[0] * pr[n0] + fc.dL0[1] * pr[n1];
                X1 = -0.5f * d - fc.Cr * v;
                Y1 = 0.5f * v;
            } else {
                const float q1 = fc.dL1[0] * pp0 + fc.dL1[1] * pp1;
                X1 = fc.wall * (fc.Cr * p1 - 0.5f * q1);
                Y1 = -fc.wall * 0.5f * p1;
            }
            float wt = 1.0f;
#pragma unroll
            for (int e = 0; e < DIM; ++e)
                if (e != a) wt *= fc.W[(n0 >> e) & 1];
            const float sd = L.sdiff[a] * wt;
#pragma unroll
            for (int ia = 0; ia < 2; ++ia) {
                float sl = fc.A[ia * 2] * pp0 + fc.A[ia * 2 + 1] * pp1;
                sl += fc.L0[ia] * X0 - fc.dL0[ia] * Y0 + fc.L1[ia] * X1 + fc.dL1[ia] * Y1;
                y[ia ? n1 : n0] += sd * sl;
            }
        }
    }
}

// one smoother step (modes of k_level) on a level in LDS, one thread per
// cell; returns after the block barrier
template <int DIM, int MODE>
__device__ void fz_step(const FusedCycle& fc, const FusedLv& L, float* lds, int din, float c1,
                        float c2) {
    constexpr int NB = 1 << DIM;
    float* x = lds + L.off;
    float* r = x + L.N;
    const float* b = x + 2 * L.N;
    float* d[2] = {x + 3 * L.N, x + 4 * L.N};
    const float* invd = x + 5 * L.N;
    const float* op = MODE == MG_RES ? x : d[din];
    float* dout = MODE == MG_RES ? d[0] : d[din ^ 1];
    for (int cell = threadIdx.x; cell < L.Nc; cell += fz_threads<DIM>()) {
        float y[NB];
        fz_apply<DIM>(fc, L, op, cell, y);
#pragma unroll
        for (int n = 0; n < NB; ++n) {
            const int i = cell * NB + n;
            const float pown = op[i];
            const float id = MODE == MG_LAST ? 0.0f : invd[i];
            if (MODE == MG_PRE1) {
                x[i] = pown;
                const float rn = b[i] - y[n];
                r[i] = rn;
                dout[i] = c1 * pown + c2 * id * rn;
            } else if (MODE == MG_STEP) {
                x[i] = x[i] + pown;
                const float rn = r[i] - y[n];
                r[i] = rn;
                dout[i] = c1 * pown + c2 * id * rn;
            } else if (MODE == MG_LAST) {
                x[i] = x[i] + pown;
                r[i] = r[i] - y[n];
            } else {   // MG_RES
                const float rn = b[i] - y[n];
                r[i] = rn;
                dout[i] = c2 * id * rn;
            }
        }
    }
    __syncthreads();
}

template <int DIM>
__global__ __launch_bounds__(fz_threads<DIM>()) void k_fused_cycle(FusedCycle fc) {
    constexpr int NT = fz_threads<DIM>();
    extern __shared__ float lds[];
    constexpr int NB = 1 << DIM;
    const int tid = threadIdx.x;
    const int m = fc.degree;
    const int nl = fc.nlev;
    // the smoothing levels' inverse diagonals, read every step, into LDS
    for (int l = 0; l < nl - 1; ++l) {
        const FusedLv& L = fc.lv[l];
        float* dst = lds + L.off + 5 * L.N;
        for (int i = tid; i < L.N; i += NT) dst[i] = L.invd[i];
    }
    // top level: right-hand side and first direction
    {
        const FusedLv& L = fc.lv[0];
        float* b = lds + L.off + 2 * L.N;
        float* d0 = lds + L.off + 3 * L.N;
        for (int i = tid; i < L.N; i += NT) {
            const float bs = fc.b_top[i];
            b[i] = bs;
            d0[i] = L.c2res * L.invd[i] * bs;
        }
        __syncthreads();
    }
    // descent
    for (int l = 0; l < nl - 1; ++l) {
        const FusedLv& L = fc.lv[l];
        fz_step<DIM, MG_PRE1>(fc, L, lds, 0, L.c1[1], L.c2[1]);
        for (int k = 2; k < m; ++k)
            fz_step<DIM, MG_STEP>(fc, L, lds, (k - 1) & 1, L.c1[k], L.c2[k]);
        fz_step<DIM, MG_LAST>(fc, L, lds, (m - 1) & 1, 0.0f, 0.0f);
        // b_c = P^T r (h-transfer), and the coarse level's first direction
        const FusedLv& C = fc.lv[l + 1];
        const bool coarsest = l + 1 == nl - 1;
        const float* rf = lds + L.off + L.N;
        float* bc = lds + C.off + 2 * C.N;
        float* dc = lds + C.off + 3 * C.N;
        for (int gid = tid; gid < C.N; gid += NT) {
            const int Cc = gid / NB, J = gid % NB;
            const int jx = J & 1, jy = (J >> 1) & 1, jz = (J >> 2) & 1;
            const int cx = Cc % C.nc[0], cy = (Cc / C.nc[0]) % C.nc[1], cz = Cc / (C.nc[0] * C.nc[1]);
            const int fnx = 2 * C.nc[0], fny = 2 * C.nc[1];
            float acc = 0.0f;
            for (int ch = 0; ch < NB; ++ch) {
                const int bx = ch & 1, by = (ch >> 1) & 1, bz = (ch >> 2) & 1;
                const int f = (2 * cx + bx) + fnx * ((2 * cy + by) + (DIM == 3 ? fny * (2 * cz + bz) : 0));
                for (int I = 0; I < NB; ++I) {
                    const int ix = I & 1, iy = (I >> 1) & 1, iz = (I >> 2) & 1;
                    float w = fc.tt.T[bx][ix][jx] * fc.tt.T[by][iy][jy];
                    if (DIM == 3) w *= fc.tt.T[bz][iz][jz];
                    acc += w * rf[f * NB + I];
                }
            }
            bc[gid] = acc;
            if (!coarsest) dc[gid] = C.c2res * lds[C.off + 5 * C.N + gid] * acc;
        }
        __syncthreads();
    }
    // coarsest: x = H^{-1} b with the FP64 inverse, one thread per row; the
    // inverse is symmetric (stored so), so thread `row` walks column `row`
    // and a wave's loads of one j are contiguous and all independent
    {
        const FusedLv& C = fc.lv[nl - 1];
        const float* b = lds + C.off + 2 * C.N;
        float* x = lds + C.off;
        for (int row = tid; row < C.N; row += NT) {
            double acc = 0.0;
#pragma unroll 8
            for (int j = 0; j < C.N; ++j) acc += fc.ainv[(size_t)j * C.N + row] * (double)b[j];
            x[row] = (float)acc;
        }
        __syncthreads();
    }
    // ascent
    int pend = -1;   // direction buffer of the level below not yet added to its x
    for (int l = nl - 2; l >= 0; --l) {
        const FusedLv& L = fc.lv[l];
        const FusedLv& C = fc.lv[l + 1];
        const float* xc = lds + C.off;
        const float* dcp = pend >= 0 ? lds + C.off + (3 + pend) * C.N : nullptr;
        float* xf = lds + L.off;
        for (int gid = tid; gid < L.N; gid += NT) {
            const int c = gid / NB, I = gid % NB;
            const int fx = c % L.nc[0], fy = (c / L.nc[0]) % L.nc[1], fzz = c / (L.nc[0] * L.nc[1]);
            const int bx = fx & 1, by = fy & 1, bz = fzz & 1;
            const int Cc = (fx >> 1) + C.nc[0] * ((fy >> 1) + (DIM == 3 ? C.nc[1] * (fzz >> 1) : 0));
            const int ix = I & 1, iy = (I >> 1) & 1, iz = (I >> 2) & 1;
            float acc = 0.0f;
            for (int J = 0; J < NB; ++J) {
                const int jx = J & 1, jy = (J >> 1) & 1, jz = (J >> 2) & 1;
                float w = fc.tt.T[bx][ix][jx] * fc.tt.T[by][iy][jy];
                if (DIM == 3) w *= fc.tt.T[bz][iz][jz];
                const int ci = Cc * NB + J;
                acc += w * (xc[ci] + (dcp ? dcp[ci] : 0.0f));
            }
            xf[gid] = xf[gid] + acc;
        }
        __syncthreads();
        fz_step<DIM, MG_RES>(fc, L, lds, 0, 0.0f, L.c2res);
        for (int k = 1; k < m; ++k)
            fz_step<DIM, MG_STEP>(fc, L, lds, (k - 1) & 1, L.c1[k], L.c2[k]);
        pend = (m - 1) & 1;
    }
    // top level out: x + d
    {
        const FusedLv& L = fc.lv[0];
        const float* x = lds + L.off;
        const float* d = lds + L.off + (3 + pend) * L.N;
        for (int i = tid; i < L.N; i += NT) fc.x_top[i] = x[i] + d[i];
    }
}

// FP64 side of flexible CG.  With `update`: alpha = sc[slot] / (sum of the Ga
// partials of p.q) (block 0 records it in sc[4], a non-positive p.q raises
// sc[6]); x += alpha p; r -= alpha q.  Always: b0 = r rounded to the level-0
// storage, d0 = c2 D^{-1} b0 (first smoother direction of the finest level),
// per-block partial sums of r.r, and after them the breakdown flag sc[6].
template <typename S>
__global__ __launch_bounds__(256) void k_mg_prep(int64_t n, int update, const double* pa, int Ga,
                                                  double* sc, int slot, double* x, double* r,
                                                  const double* p, const double* q, S* b0,
                                                  S* d0, const float* invd, float c2,
                                                  double* partial) {
    using T = Sto<S>;
    __shared__ double s_alpha;
    double alpha = 0.0;
    if (update) {
        double pq = 0.0;
        for (int k = threadIdx.x; k < Ga; k += 256) pq += pa[k];
        pq = red::block_sum(pq);
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
        alpha = s_alpha;
    }
    double rr = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        double ri = r[i];
        if (update) {
            x[i] += alpha * p[i];
            ri -= alpha * q[i];
            r[i] = ri;
        }
        rr += ri * ri;
        const float bs = T::put(b0, i, (float)ri);
        T::put(d0, i, c2 * invd[i] * bs);
    }
    rr = red::block_sum(rr);
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = rr;
        // the breakdown flag travels with the partials (one host copy)
        if (blockIdx.x == 0) partial[gridDim.x] = sc[6];
    }
}

// ---- the constant mode of the BF16 cycle -----------------------------------------
// K 1 = 0, so H 1 = alpha M 1 exactly and H^{-1} r has the constant component
// (1.r) / (alpha 1.M1) with m.z = (1.r) / alpha (m = M 1); the rest is
// m-orthogonal.  Rounding the finest level's vectors to bf16 injects a
// constant component of relative size 2^-9 that the cycle, an approximate
// inverse, multiplies by ~1/alpha (alpha = 1/(c^2 beta^2 dt^2) is small):
// z then carries a spurious constant.  The fix replaces z's m-weighted
// constant by the exact one, z += gamma 1 with
//   gamma = (1.r) / (alpha 1.m) - (m.z) / (1.m),
// and recomputes the z.r and z.q partials of flexible CG.

// partials of 1.r, 1.q (q may be null) and m.z
__global__ __launch_bounds__(256) void k_defl_sums(int64_t n, const double* __restrict__ r,
                                                    const double* __restrict__ q,
                                                    const double* __restrict__ m,
                                                    const double* __restrict__ z,
                                                    double* __restrict__ partial) {
    double sr = 0.0, sq = 0.0, mz = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        sr += r[i];
        if (q) sq += q[i];
        if (z) mz += m[i] * z[i];
    }
    sr = red::block_sum(sr);
    sq = red::block_sum(sq);
    mz = red::block_sum(mz);
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = sr;
        partial[gridDim.x + blockIdx.x] = sq;
        partial[2 * gridDim.x + blockIdx.x] = mz;
    }
}

// every block sums the G partials of k_defl_sums in the same order, forms
// gamma, adds it to z and writes its partials of z.r and z.q (k_mg_beta's
// layout: G2 blocks of this kernel)
__global__ __launch_bounds__(256) void k_defl_apply(int64_t n, const double* __restrict__ sums, int G,
                                                     double alpha, double mtot,
                                                     const double* __restrict__ r,
                                                     const double* __restrict__ q,
                                                     double* __restrict__ z,
                                                     double* __restrict__ partial) {
    __shared__ double s_g;
    double sr = 0.0, mz = 0.0;
    for (int k = threadIdx.x; k < G; k += 256) {
        sr += sums[k];
        mz += sums[2 * G + k];
    }
    sr = red::block_sum(sr);
    mz = red::block_sum(mz);
    if (threadIdx.x == 0) s_g = sr / (alpha * mtot) - mz / mtot;
    __syncthreads();
    const double g = s_g;
    double zr = 0.0, zq = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const double zi = z[i] + g;
        z[i] = zi;
        zr += zi * r[i];
        if (q) zq += zi * q[i];
    }
    zr = red::block_sum(zr);
    zq = red::block_sum(zq);
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = zr;
        partial[gridDim.x + blockIdx.x] = zq;
    }
}

// start of a BF16 solve: the exact constant mode of the residual moved into
// x, x += g 1 and r -= g alpha m with g = (1.r) / (alpha 1.m) (H 1 = alpha m)
__global__ __launch_bounds__(256) void k_defl_start(int64_t n, const double* __restrict__ sums, int G,
                                                     double alpha, double mtot,
                                                     const double* __restrict__ m,
                                                     double* __restrict__ x, double* __restrict__ r) {
    __shared__ double s_g;
    double sr = 0.0;
    for (int k = threadIdx.x; k < G; k += 256) sr += sums[k];
    sr = red::block_sum(sr);
    if (threadIdx.x == 0) s_g = sr / (alpha * mtot);
    __syncthreads();
    const double g = s_g;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        x[i] += g;
        r[i] -= g * alpha * m[i];
    }
}

// beta of flexible CG from the z.r and z.q partials of the last smoother step:
// beta = -alpha z.q / (z.r)_old (0 on the first step); sc[slot] = z.r.  A
// non-positive or non-finite z.r (preconditioner not positive) raises sc[6].
__global__ __launch_bounds__(256) void k_mg_beta(const double* partial, int G, double* sc,
                                                  int first, int slot, int slot_prev) {
    double zr = 0.0, zq = 0.0;
    for (int k = threadIdx.x; k < G; k += 256) {
        zr += partial[k];
        zq += partial[G + k];
    }
    zr = red::block_sum(zr);
    zq = red::block_sum(zq);
    if (threadIdx.x == 0) {
        sc[5] = first ? 0.0 : -sc[4] * zq / sc[slot_prev];
        sc[slot] = zr;
        if (!(zr > 0.0) || !isfinite(zr)) sc[6] = 1.0;
    }
}

// b0 = s v_comp, d0 = c2 D^{-1} b0 (s = scale, times *sc_dev when given);
// v in the velocity layout [cell][component][node], b0 and d0 one scalar
// field [cell][node].
__global__ __launch_bounds__(256) void k_vel_prep(int64_t n, int nb, int dim, int comp,
                                                   const double* __restrict__ v,
                                                   const double* __restrict__ sc_dev, double scale,
                                                   float* __restrict__ b0, float* __restrict__ d0,
                                                   const float* __restrict__ invd, float c2) {
    const double s = sc_dev ? scale * sc_dev[0] : scale;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const int64_t cell = i / nb;
        const int nd = (int)(i - cell * nb);
        const float bs = (float)(s * v[(cell * dim + comp) * nb + nd]);
        b0[i] = bs;
        d0[i] = c2 * invd[i] * bs;
    }
}

__global__ __launch_bounds__(256) void k_mul3(int64_t n, const double* a, const double* b,
                                               double* out) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        out[i] = a[i] * b[i];
}

__global__ __launch_bounds__(256) void k_unit(int64_t n, int64_t j, double* out) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        out[i] = i == j ? 1.0 : 0.0;
}

__global__ __launch_bounds__(256) void k_fill(int64_t n, double v, double* out) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        out[i] = v;
}

__global__ __launch_bounds__(256) void k_inv_sqrt_to(int64_t n, const double* d, double* out,
                                                      float* invf) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        out[i] = 1.0 / sqrt(d[i]);
        invf[i] = (float)(1.0 / d[i]);
    }
}

inline unsigned nblk(int64_t work, int per) { return (unsigned)((work + per - 1) / per); }
inline unsigned gs_grid(int64_t n) {
    const int64_t g = (n + 255) / 256;
    return (unsigned)(g < 1024 ? (g > 0 ? g : 1) : 1024);
}

}  // namespace

// ---- launchers -------------------------------------------------------------------
#define TBDG_LV_DISPATCH(dim, np, FN)                                                    \
    do {                                                                                  \
        if ((dim) == 2 && (np) == 2) { FN(2, 2); }                                        \
        else if ((dim) == 2 && (np) == 3) { FN(2, 3); }                                   \
        else if ((dim) == 2 && (np) == 4) { FN(2, 4); }                                   \
        else if ((dim) == 2 && (np) == 5) { FN(2, 5); }                                   \
        else if ((dim) == 2 && (np) == 6) { FN(2, 6); }                                   \
        else if ((dim) == 3 && (np) == 2) { FN(3, 2); }                                   \
        else if ((dim) == 3 && (np) == 3) { FN(3, 3); }                                   \
        else if ((dim) == 3 && (np) == 4) { FN(3, 4); }                                   \
        else throw Error(TBDG_EUNSUPPORTED, "unsupported multigrid level");               \
    } while (0)

template <typename S>
int launch_level_step(hipStream_t st, int dim, const MGLevel& L, int stage, int mode, float c1,
                      float c2, const S* dop, S* x, S* r, const S* b, S* dout, double* z,
                      const double* r64, const double* q64, double* partial, int zs) {
    int G = 0;
    if (zs <= 0) zs = (int)(L.N / L.Nc);
    const float cm = L.tf.cm[stage];
    const float* invd = L.invd[stage];
#define K_(D, NP, MODE)                                                                    \
    hipLaunchKernelGGL((k_level<D, NP, S, MODE>), dim3(G), dim3(256), 0, st, L.geom,       \
                       L.lgeom, L.tf, cm, c1, c2, dop, x, r, b, invd, dout, (int)L.Nc, z,  \
                       r64, q64, partial, zs)
#define L_(D, NP)                                                                          \
    {                                                                                      \
        G = (int)nblk(L.Nc, FaceLay<D, NP>::CPB);                                          \
        switch (mode) {                                                                    \
            case MG_PRE1: K_(D, NP, MG_PRE1); break;                                         \
            case MG_STEP: K_(D, NP, MG_STEP); break;                                         \
            case MG_LAST: K_(D, NP, MG_LAST); break;                                         \
            case MG_RES: K_(D, NP, MG_RES); break;                                           \
            default: K_(D, NP, MG_ZFIN); break;                                             \
        }                                                                                  \
    }
    TBDG_LV_DISPATCH(dim, L.np, L_);
#undef L_
#undef K_
    TBDG_HIP(hipGetLastError());
    return G;
}
template int launch_level_step<float>(hipStream_t, int, const MGLevel&, int, int, float, float,
                                      const float*, float*, float*, const float*, float*,
                                      double*, const double*, const double*, double*, int);
template int launch_level_step<uint16_t>(hipStream_t, int, const MGLevel&, int, int, float,
                                         float, const uint16_t*, uint16_t*, uint16_t*,
                                         const uint16_t*, uint16_t*, double*, const double*,
                                         const double*, double*, int);

int level_blocks(int dim, const MGLevel& L) {
    int G = 0;
#define L_(D, NP) G = (int)nblk(L.Nc, FaceLay<D, NP>::CPB);
    TBDG_LV_DISPATCH(dim, L.np, L_);
#undef L_
    return G;
}

template <typename S>
void launch_restrict(hipStream_t st, int dim, const MGLevel& F, const MGLevel& C, int stage,
                     float c2, const S* rf, bool with_d0) {
    float* d0 = with_d0 ? C.d[0] : nullptr;
    const float* invd = with_d0 ? C.invd[stage] : nullptr;
    const unsigned G = nblk(C.N, 256);
#define L_(D, NF)                                                                          \
    {                                                                                      \
        if (F.transfer == 1)                                                               \
            hipLaunchKernelGGL((k_restrict<D, NF, S, 0>), dim3(G), dim3(256), 0, st, F.tt,  \
                               rf, C.b, d0, invd, c2, C.geom.nc[0], C.geom.nc[1],          \
                               C.geom.nc[2], (int)C.Nc);                                    \
        else                                                                               \
            hipLaunchKernelGGL((k_restrict<D, 2, S, 1>), dim3(G), dim3(256), 0, st, F.tt,   \
                               rf, C.b, d0, invd, c2, C.geom.nc[0], C.geom.nc[1],          \
                               C.geom.nc[2], (int)C.Nc);                                    \
    }
    TBDG_LV_DISPATCH(dim, F.np, L_);
#undef L_
    TBDG_HIP(hipGetLastError());
}
template void launch_restrict<float>(hipStream_t, int, const MGLevel&, const MGLevel&, int, float,
                                     const float*, bool);
template void launch_restrict<uint16_t>(hipStream_t, int, const MGLevel&, const MGLevel&, int,
                                        float, const uint16_t*, bool);

template <typename S>
void launch_prolong(hipStream_t st, int dim, const MGLevel& F, const MGLevel& C, S* xf,
                    const float* dc) {
    const unsigned G = nblk(F.N, 256);
#define L_(D, NF)                                                                          \
    {                                                                                      \
        if (F.transfer == 1)                                                               \
            hipLaunchKernelGGL((k_prolong<D, NF, S, 0>), dim3(G), dim3(256), 0, st, F.tt,   \
                               xf, C.x, dc, F.geom.nc[0], F.geom.nc[1], (int)F.Nc);        \
        else                                                                               \
            hipLaunchKernelGGL((k_prolong<D, 2, S, 1>), dim3(G), dim3(256), 0, st, F.tt,    \
                               xf, C.x, dc, F.geom.nc[0], F.geom.nc[1], (int)F.Nc);        \
    }
    TBDG_LV_DISPATCH(dim, F.np, L_);
#undef L_
    TBDG_HIP(hipGetLastError());
}
template void launch_prolong<float>(hipStream_t, int, const MGLevel&, const MGLevel&, float*,
                                    const float*);
template void launch_prolong<uint16_t>(hipStream_t, int, const MGLevel&, const MGLevel&,
                                       uint16_t*, const float*);

void launch_coarse(hipStream_t st, const double* Ainv, const float* b, float* x, int n) {
    hipLaunchKernelGGL(k_coarse, dim3(nblk(n, 4)), dim3(256), 0, st, Ainv, b, x, n);
    TBDG_HIP(hipGetLastError());
}

template <typename S>
int launch_mg_prep(hipStream_t st, int64_t n, int update, const double* pa, int Ga, double* sc,
                   int slot, double* x, double* r, const double* p, const double* q, S* b0, S* d0,
                   const float* invd, float c2, double* partial) {
    // at most 1024 partials (gs_grid's cap): the host adds them from its
    // 2048-entry pinned buffer; 1024 blocks keep four per CU streaming
    const unsigned G = gs_grid(n);
    hipLaunchKernelGGL((k_mg_prep<S>), dim3(G), dim3(256), 0, st, n, update, pa, Ga, sc, slot, x,
                       r, p, q, b0, d0, invd, c2, partial);
    TBDG_HIP(hipGetLastError());
    return (int)G;
}
template int launch_mg_prep<float>(hipStream_t, int64_t, int, const double*, int, double*, int,
                                   double*, double*, const double*, const double*, float*, float*,
                                   const float*, float, double*);
template int launch_mg_prep<uint16_t>(hipStream_t, int64_t, int, const double*, int, double*, int,
                                      double*, double*, const double*, const double*, uint16_t*,
                                      uint16_t*, const float*, float, double*);

int launch_deflate(hipStream_t st, int64_t n, double alpha, double mtot, const double* m,
                   const double* r, const double* q, double* z, double* sums, double* zpart,
                   int max_blocks) {
    const unsigned G = gs_grid(n) < 256u ? gs_grid(n) : 256u;
    hipLaunchKernelGGL(k_defl_sums, dim3(G), dim3(256), 0, st, n, r, q, m, z, sums);
    unsigned G2 = gs_grid(n);
    if ((int)G2 > max_blocks) G2 = (unsigned)max_blocks;
    hipLaunchKernelGGL(k_defl_apply, dim3(G2), dim3(256), 0, st, n, sums, (int)G, alpha, mtot, r, q, z,
                       zpart);
    TBDG_HIP(hipGetLastError());
    return (int)G2;
}

void launch_deflate_start(hipStream_t st, int64_t n, double alpha, double mtot, const double* m,
                          double* x, double* r, double* sums) {
    const unsigned G = gs_grid(n) < 256u ? gs_grid(n) : 256u;
    hipLaunchKernelGGL(k_defl_sums, dim3(G), dim3(256), 0, st, n, r, (const double*)nullptr, m,
                       (const double*)nullptr, sums);
    hipLaunchKernelGGL(k_defl_start, dim3(gs_grid(n)), dim3(256), 0, st, n, sums, (int)G, alpha, mtot, m,
                       x, r);
    TBDG_HIP(hipGetLastError());
}

void launch_mg_beta(hipStream_t st, const double* partial, int G, double* sc, int first, int slot,
                    int slot_prev) {
    hipLaunchKernelGGL(k_mg_beta, dim3(1), dim3(256), 0, st, partial, G, sc, first, slot,
                       slot_prev);
    TBDG_HIP(hipGetLastError());
}

void launch_fused_cycle(hipStream_t st, int dim, const FusedCycle& fc, size_t lds) {
    if (dim == 2)
        hipLaunchKernelGGL(k_fused_cycle<2>, dim3(1), dim3(fz_threads<2>()), lds, st, fc);
    else
        hipLaunchKernelGGL(k_fused_cycle<3>, dim3(1), dim3(fz_threads<3>()), lds, st, fc);
    TBDG_HIP(hipGetLastError());
}

size_t fused_lds_limit(int dim) {
    int dev = 0, v = 0;
    TBDG_HIP(hipGetDevice(&dev));
    TBDG_HIP(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    const void* fn = dim == 2 ? (const void*)k_fused_cycle<2> : (const void*)k_fused_cycle<3>;
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, v) != hipSuccess) {
        (void)hipGetLastError();
        v = 65536 < v ? 65536 : v;
    }
    return (size_t)v;
}

void launch_vel_prep(hipStream_t st, int64_t Nc, int nb, int dim, int comp, const double* v,
                     const double* sc_dev, double scale, float* b0, float* d0, const float* invd,
                     float c2) {
    const int64_t n = Nc * nb;
    hipLaunchKernelGGL(k_vel_prep, dim3(gs_grid(n)), dim3(256), 0, st, n, nb, dim, comp, v, sc_dev,
                       scale, b0, d0, invd, c2);
    TBDG_HIP(hipGetLastError());
}

void vec_mul(hipStream_t st, int64_t n, const double* a, const double* b, double* out) {
    hipLaunchKernelGGL(k_mul3, dim3(gs_grid(n)), dim3(256), 0, st, n, a, b, out);
    TBDG_HIP(hipGetLastError());
}

void vec_fill(hipStream_t st, int64_t n, double v, double* out) {
    hipLaunchKernelGGL(k_fill, dim3(gs_grid(n)), dim3(256), 0, st, n, v, out);
    TBDG_HIP(hipGetLastError());
}

void vec_unit(hipStream_t st, int64_t n, int64_t j, double* out) {
    hipLaunchKernelGGL(k_unit, dim3(gs_grid(n)), dim3(256), 0, st, n, j, out);
    TBDG_HIP(hipGetLastError());
}

void vec_inv_sqrt(hipStream_t st, int64_t n, const double* d, double* out, float* invf) {
    hipLaunchKernelGGL(k_inv_sqrt_to, dim3(gs_grid(n)), dim3(256), 0, st, n, d, out, invf);
    TBDG_HIP(hipGetLastError());
}

}  // namespace trbdg
