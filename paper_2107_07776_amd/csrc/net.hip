// Kernels of the learned pressure-guess network: 3x3x3 circular convolutions
// as implicit GEMMs on the bf16 matrix cores (v_mfma_f32_16x16x32_bf16, FP32
// accumulation), the weight gradient with FP32 accumulation, MSE, Adam and the
// layout conversions.
//
// Activations are stored channel-last in bf16, [voxel][channel] with the
// channel count a multiple of 8, voxels lexicographic (x fastest) per sample
// and samples one after the other.  A convolution is the GEMM
//   Y[co][v] = sum_{s, j} Wp[s][co][j] * X[nbr(v, k(s))][8 cg(s) + j]
// over "slots" s = k * CG + cg (k = 3x3x3 offset, cg = group of 8 input
// channels, CG = channels / 8), four slots per MFMA (K = 32).  The matrix
// core's K order is the same for both operands, so each lane loads the 8
// consecutive channels of one slot for the weights (rows = output channels)
// and for the activations (columns = voxels).
#include <hip/hip_runtime.h>

#include "internal.hpp"
#include "reduce.hpp"

namespace trbdg {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ inline uint16_t f2bf(float v) {
    const unsigned u = __float_as_uint(v);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
    return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__device__ inline float bf2f(uint16_t h) { return __uint_as_float((unsigned)h << 16); }

constexpr int round4(int x) { return (x + 3) / 4 * 4; }

// Voxel index of the neighbour at offset k (0..26, dz outer, dx inner) of
// the voxel with coordinates (x, y, z) in sample b, periodic wrap.
struct VoxNbr {
    // wrapped by arithmetic, not through a table: a per-lane table index
    // would put the table in private (scratch) memory
    int base, x, y, z, nx, ny, nz;
    __device__ VoxNbr(int v, const NetGeo& g) : nx(g.nx), ny(g.ny), nz(g.nz) {
        const int b = v / g.nvox, r = v - b * g.nvox;
        x = r % g.nx;
        y = (r / g.nx) % g.ny;
        z = r / (g.nx * g.ny);
        base = b * g.nvox;
    }
    __device__ static int wrap(int c, int n) { return c < 0 ? c + n : (c >= n ? c - n : c); }
    __device__ int at(int k) const {
        const int zz = wrap(z + k / 9 - 1, nz), yy = wrap(y + (k / 3) % 3 - 1, ny),
                  xx = wrap(x + k % 3 - 1, nx);
        return base + (zz * ny + yy) * nx + xx;
    }
};

// MODE 0: hidden layer, Y = bf16(relu(acc + bias)), [v][COUT]
// MODE 1: last layer (output channels 0 .. nout-1 <= 3 of a 16-row tile),
//         y = acc + bias, FP32 [b][nout][voxel of the sample]
// MODE 2: input gradient, Y = bf16(acc * (mask > 0)), mask [v][COUT] bf16
template <int CIN, int COUT, int MODE>
__global__ __launch_bounds__(256) void k_conv_mfma(NetGeo g, const uint16_t* __restrict__ X,
                                                    const uint16_t* __restrict__ Wp,
                                                    const float* __restrict__ bias,
                                                    uint16_t* __restrict__ Yb,
                                                    float* __restrict__ Yf,
                                                    const uint16_t* __restrict__ mask, int nout) {
    constexpr int CG = CIN / 8;
    constexpr int S = round4(27 * CG);
    constexpr int CT = COUT / 16;
    constexpr int STRIPS = 4;                 // strips of 16 voxels per wave
    __shared__ bf16x8 s_w[S * COUT];
    const int tid = threadIdx.x;
    {
        const bf16x8* src = reinterpret_cast<const bf16x8*>(Wp);
        for (int i = tid; i < S * COUT; i += 256) s_w[i] = src[i];
    }
    __syncthreads();
    const int wave = tid / 64, lane = tid % 64;
    const int col = lane % 16, grp = lane / 16;
    const int total = g.nvox * g.B;
    for (int st = 0; st < STRIPS; ++st) {
        const int v0 = ((blockIdx.x * 4 + wave) * STRIPS + st) * 16;
        if (v0 >= total) break;
        const int v = v0 + col;
        const VoxNbr nb(v < total ? v : total - 1, g);
        f32x4 acc[CT];
#pragma unroll
        for (int c = 0; c < CT; ++c) acc[c] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        for (int t = 0; t < S / 4; ++t) {
            const int s = 4 * t + grp;
            const int k = s / CG < 27 ? s / CG : 26;     // padded slots carry zero weights
            const int cg = s % CG;
            const bf16x8 bfrag = *reinterpret_cast<const bf16x8*>(X + (size_t)nb.at(k) * CIN + cg * 8);
#pragma unroll
            for (int c = 0; c < CT; ++c) {
                const bf16x8 afrag = s_w[s * COUT + c * 16 + col];
                acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afrag, bfrag, acc[c], 0, 0, 0);
            }
        }
        if (v >= total) continue;
        if (MODE == 1) {
            // lanes of group 0 hold rows 0..3 of the tile: the output channels
            if (grp == 0) {
                const int b = v / g.nvox, r = v - b * g.nvox;
#pragma unroll
                for (int o = 0; o < 4; ++o)
                    if (o < nout) Yf[((size_t)b * nout + o) * g.nvox + r] = acc[0][o] + bias[o];
            }
            continue;
        }
#pragma unroll
        for (int c = 0; c < CT; ++c) {
            const int co = c * 16 + 4 * grp;
            uint16_t h[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                float val = acc[c][r];
                if (MODE == 0) val = fmaxf(val + bias[co + r], 0.0f);
                else val = bf2f(mask[(size_t)v * COUT + co + r]) > 0.0f ? val : 0.0f;
                h[r] = f2bf(val);
            }
            uint2 pk;
            pk.x = (unsigned)h[0] | ((unsigned)h[1] << 16);
            pk.y = (unsigned)h[2] | ((unsigned)h[3] << 16);
            *reinterpret_cast<uint2*>(Yb + (size_t)v * COUT + co) = pk;
        }
    }
}

// Weight gradient, FP32 accumulation: for the block's rows of voxels
//   partial[blk][(co * CIN + ci) * 27 + k] = sum_v dY[v][co] * X[nbr(v, k)][ci]
//   partial[blk][COUT * CIN * 27 + co]     = sum_v dY[v][co]
// Each thread owns (k, ci) pairs and all output channels; one row (nx
// voxels) of dY and the 3x3 neighbouring rows of X are staged in LDS.
template <int CIN, int COUT, int DYS>
__global__ __launch_bounds__(256) void k_conv_wgrad(NetGeo g, const uint16_t* __restrict__ X,
                                                     const uint16_t* __restrict__ dY,
                                                     float* __restrict__ partial, int rows_per_block) {
    constexpr int PAIRS = 27 * CIN;
    constexpr int PT = (PAIRS + 255) / 256;
    constexpr int NP = COUT * CIN * 27 + COUT;
    extern __shared__ float s_dyn[];
    float* s_dy = s_dyn;                                   // [nx][COUT]
    uint16_t* s_x = reinterpret_cast<uint16_t*>(s_dy + g.nx * COUT);   // [9][nx][CIN]
    const int tid = threadIdx.x;
    float acc[PT][COUT];
    float bacc = 0.0f;
#pragma unroll
    for (int p = 0; p < PT; ++p)
#pragma unroll
        for (int co = 0; co < COUT; ++co) acc[p][co] = 0.0f;
    const int rows = g.B * g.ny * g.nz;
    const int r0 = blockIdx.x * rows_per_block;
    for (int row = r0; row < r0 + rows_per_block && row < rows; ++row) {
        const int b = row / (g.ny * g.nz), rr = row % (g.ny * g.nz);
        const int y = rr % g.ny, z = rr / g.ny;
        const size_t vrow = (size_t)b * g.nvox + (size_t)rr * g.nx;
        __syncthreads();
        for (int i = tid; i < g.nx * COUT; i += 256) {
            const int x = i / COUT, co = i % COUT;
            s_dy[i] = bf2f(dY[(vrow + x) * DYS + co]);
        }
        for (int i = tid; i < 9 * g.nx * CIN; i += 256) {
            const int q = i / (g.nx * CIN), rem = i % (g.nx * CIN);
            const int dz = q / 3 - 1, dy = q % 3 - 1;
            const int zz = (z + dz + g.nz) % g.nz, yy = (y + dy + g.ny) % g.ny;
            s_x[i] = X[((size_t)b * g.nvox + ((size_t)zz * g.ny + yy) * g.nx) * CIN + rem];
        }
        __syncthreads();
        for (int x = 0; x < g.nx; ++x) {
            const float* dyx = s_dy + x * COUT;
#pragma unroll
            for (int p = 0; p < PT; ++p) {
                const int pair = tid + p * 256;
                if (pair >= PAIRS) break;
                const int k = pair / CIN, ci = pair % CIN;
                const int dx = k % 3 - 1, q = k / 3;     // q = (dz + 1) * 3 + (dy + 1)
                int xx = x + dx;
                xx = xx < 0 ? xx + g.nx : (xx >= g.nx ? xx - g.nx : xx);
                const float xv = bf2f(s_x[(q * g.nx + xx) * CIN + ci]);
#pragma unroll
                for (int co = 0; co < COUT; ++co) acc[p][co] += dyx[co] * xv;
            }
            if (tid < COUT) bacc += dyx[tid];
        }
    }
    float* out = partial + (size_t)blockIdx.x * NP;
#pragma unroll
    for (int p = 0; p < PT; ++p) {
        const int pair = tid + p * 256;
        if (pair >= PAIRS) break;
        const int k = pair / CIN, ci = pair % CIN;
#pragma unroll
        for (int co = 0; co < COUT; ++co) out[(co * CIN + ci) * 27 + k] = acc[p][co];
    }
    if (tid < COUT) out[COUT * CIN * 27 + tid] = bacc;
}

// grad[i] += sum_b partial[b][i] (fixed order), scattered into the master
// layout: W[co][ci < cin_real][k] at w_off, b[co] at b_off.
__global__ __launch_bounds__(256) void k_wgrad_reduce(const float* partial, int G, int cout,
                                                      int cin, int cin_real, float* grad, int64_t w_off,
                                                      int64_t b_off) {
    const int np = cout * cin * 27 + cout;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= np) return;
    float s = 0.0f;
    for (int b = 0; b < G; ++b) s += partial[(size_t)b * np + i];
    if (i < cout * cin * 27) {
        const int co = i / (cin * 27), ci = (i / 27) % cin, k = i % 27;
        if (ci < cin_real) grad[w_off + ((int64_t)co * cin_real + ci) * 27 + k] += s;
    } else {
        grad[b_off + (i - cout * cin * 27)] += s;
    }
}

// Forward pack: Wp[s][co][j] = W[co][ci][k] with s = k * CG + cg, ci = 8 cg + j
// (zero beyond the real channels and for padded slots); W at theta + w_off in
// [cout_real][cin_real][27] order.
__global__ __launch_bounds__(256) void k_pack_fwd(const float* theta, int64_t w_off, int cout_real,
                                                  int cin_real, int cin, int cout, int S,
                                                  uint16_t* Wp) {
    const int n = S * cout * 8;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int j = i % 8, co = (i / 8) % cout, s = i / (8 * cout);
    const int CG = cin / 8;
    const int k = s / CG, ci = (s % CG) * 8 + j;
    float v = 0.0f;
    if (k < 27 && co < cout_real && ci < cin_real) v = theta[w_off + ((int64_t)co * cin_real + ci) * 27 + k];
    Wp[i] = f2bf(v);
}

// Input-gradient pack: the transposed, flipped kernel as a forward pack with
// input channels = the layer's outputs (cin2 = cout padded to 8) and output
// channels = the layer's inputs: Wt[s][ci][j] = W[co = 8 cg + j][ci][26 - k].
__global__ __launch_bounds__(256) void k_pack_bwd(const float* theta, int64_t w_off, int cout_real,
                                                  int cin_real, int cin2, int S, uint16_t* Wt) {
    const int n = S * cin_real * 8;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int j = i % 8, ci = (i / 8) % cin_real, s = i / (8 * cin_real);
    const int CG = cin2 / 8;
    const int k = s / CG, co = (s % CG) * 8 + j;
    float v = 0.0f;
    if (k < 27 && co < cout_real) v = theta[w_off + ((int64_t)co * cin_real + ci) * 27 + (26 - k)];
    Wt[i] = f2bf(v);
}

__global__ __launch_bounds__(256) void k_copy_bias(const float* theta, int64_t b_off, int n, float* b) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) b[i] = theta[b_off + i];
}

// fp32 [B][C][nvox] -> bf16 [B*nvox][CP] (channels beyond C zero)
__global__ __launch_bounds__(256) void k_to_channel_last(const float* x, int B, int C, int nvox, int CP,
                                                         uint16_t* out) {
    const int64_t n = (int64_t)B * nvox * CP;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const int c = (int)(i % CP);
        const int64_t v = i / CP;
        const int b = (int)(v / nvox), r = (int)(v % nvox);
        out[i] = c < C ? f2bf(x[((int64_t)b * C + c) * nvox + r]) : (uint16_t)0;
    }
}

// Quadratic loss of the guess's blend per cell (y0, y1 at yhat[b][0..1][c],
// Gram data at gram[b][0..5][c]): l = ee - 2 (y0 r1 + y1 r2) + y0^2 g11
// + 2 y0 y1 g12 + y1^2 g22, dy = dl/dy / (B n); per-block partial sums of l
__global__ __launch_bounds__(256) void k_quad_loss(const float* yhat, const float* gram, int64_t n, int B,
                                                   float* dy, double* partial) {
    const int64_t total = n * B;
    const double inv = 1.0 / (double)total;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256) {
        const int64_t b = i / n, c = i - b * n;
        const float* yb = yhat + b * 2 * n;
        const float* gb = gram + b * 6 * n;
        const double y0 = yb[c], y1 = yb[n + c];
        const double g11 = gb[c], g12 = gb[n + c], g22 = gb[2 * n + c];
        const double r1 = gb[3 * n + c], r2 = gb[4 * n + c], ee = gb[5 * n + c];
        acc += ee - 2.0 * (y0 * r1 + y1 * r2) + y0 * y0 * g11 + 2.0 * y0 * y1 * g12 + y1 * y1 * g22;
        float* db = dy + b * 2 * n;
        db[c] = (float)(2.0 * (y0 * g11 + y1 * g12 - r1) * inv);
        db[n + c] = (float)(2.0 * (y0 * g12 + y1 * g22 - r2) * inv);
    }
    acc = red::block_sum(acc);
    if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

// MSE: dy = 2 (yhat - y) / n, per-block partial sums of (yhat - y)^2
__global__ __launch_bounds__(256) void k_mse(const float* yhat, const float* y, int64_t n, float* dy,
                                             double* partial) {
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const float d = yhat[i] - y[i];
        dy[i] = 2.0f * d / (float)n;
        acc += (double)d * d;
    }
    acc = red::block_sum(acc);
    if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

__global__ __launch_bounds__(256) void k_adam(int64_t n, float* theta, const float* g, float* m,
                                              float* v, float lr, float b1, float b2, float eps,
                                              float c1, float c2) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        theta[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

inline unsigned nb256(int64_t n) { return (unsigned)((n + 255) / 256); }
inline unsigned gs(int64_t n) {
    const int64_t g = (n + 255) / 256;
    return (unsigned)(g < 2048 ? (g > 0 ? g : 1) : 2048);
}

}  // namespace

// ---- launchers ----------------------------------------------------------------------
void net_conv(hipStream_t st, const NetGeo& g, int cin, int cout, int mode, const uint16_t* X,
              const uint16_t* Wp, const float* bias, uint16_t* Yb, float* Yf, const uint16_t* mask,
              int nout) {
    if (mode == 1 && (nout < 1 || nout > 4)) throw Error(TBDG_EINVAL, "last layer writes 1..4 outputs");
    // 4 waves x 4 strips x 16 voxels per block
    const unsigned G = (unsigned)((g.nvox * (int64_t)g.B + 255) / 256);
#define K_(CI, CO, M) hipLaunchKernelGGL((k_conv_mfma<CI, CO, M>), dim3(G), dim3(256), 0, st, g, X, Wp, bias, Yb, Yf, mask, nout)
    if (cin == 8 && cout == 32 && mode == 0) K_(8, 32, 0);
    else if (cin == 32 && cout == 32 && mode == 0) K_(32, 32, 0);
    else if (cin == 32 && cout == 16 && mode == 1) K_(32, 16, 1);
    else if (cin == 8 && cout == 32 && mode == 2) K_(8, 32, 2);
    else if (cin == 32 && cout == 32 && mode == 2) K_(32, 32, 2);
    else throw Error(TBDG_EUNSUPPORTED, "unsupported convolution shape");
#undef K_
    TBDG_HIP(hipGetLastError());
}

int net_wgrad(hipStream_t st, const NetGeo& g, int cin, int cout, int dys, const uint16_t* X,
              const uint16_t* dY, float* partial, int rows_per_block) {
    const int rows = g.B * g.ny * g.nz;
    const unsigned G = (unsigned)((rows + rows_per_block - 1) / rows_per_block);
    const size_t lds = sizeof(float) * g.nx * cout + sizeof(uint16_t) * 9 * g.nx * cin;
#define K_(CI, CO, D) hipLaunchKernelGGL((k_conv_wgrad<CI, CO, D>), dim3(G), dim3(256), lds, st, g, X, dY, partial, rows_per_block)
    if (cin == 8 && cout == 32 && dys == 32) K_(8, 32, 32);
    else if (cin == 32 && cout == 32 && dys == 32) K_(32, 32, 32);
    else if (cin == 32 && cout == 1 && dys == 8) K_(32, 1, 8);
    else if (cin == 32 && cout == 2 && dys == 8) K_(32, 2, 8);
    else throw Error(TBDG_EUNSUPPORTED, "unsupported weight-gradient shape");
#undef K_
    TBDG_HIP(hipGetLastError());
    return (int)G;
}

void net_wgrad_reduce(hipStream_t st, const float* partial, int G, int cout, int cin, int cin_real,
                      float* grad, int64_t w_off, int64_t b_off) {
    const int np = cout * cin * 27 + cout;
    hipLaunchKernelGGL(k_wgrad_reduce, dim3(nb256(np)), dim3(256), 0, st, partial, G, cout, cin,
                       cin_real, grad, w_off, b_off);
    TBDG_HIP(hipGetLastError());
}

void net_pack_fwd(hipStream_t st, const float* theta, int64_t w_off, int cout_real, int cin_real,
                  int cin, int cout, int S, uint16_t* Wp) {
    hipLaunchKernelGGL(k_pack_fwd, dim3(nb256((int64_t)S * cout * 8)), dim3(256), 0, st, theta, w_off,
                       cout_real, cin_real, cin, cout, S, Wp);
    TBDG_HIP(hipGetLastError());
}

void net_pack_bwd(hipStream_t st, const float* theta, int64_t w_off, int cout_real, int cin_real,
                  int cin2, int S, uint16_t* Wt) {
    hipLaunchKernelGGL(k_pack_bwd, dim3(nb256((int64_t)S * cin_real * 8)), dim3(256), 0, st, theta,
                       w_off, cout_real, cin_real, cin2, S, Wt);
    TBDG_HIP(hipGetLastError());
}

void net_copy_bias(hipStream_t st, const float* theta, int64_t b_off, int n, float* b) {
    hipLaunchKernelGGL(k_copy_bias, dim3(nb256(n)), dim3(256), 0, st, theta, b_off, n, b);
    TBDG_HIP(hipGetLastError());
}

void net_to_channel_last(hipStream_t st, const float* x, int B, int C, int nvox, int CP, uint16_t* out) {
    hipLaunchKernelGGL(k_to_channel_last, dim3(gs((int64_t)B * nvox * CP)), dim3(256), 0, st, x, B, C,
                       nvox, CP, out);
    TBDG_HIP(hipGetLastError());
}

int net_quad_loss(hipStream_t st, const float* yhat, const float* gram, int64_t n, int B, float* dy,
                  double* partial) {
    const unsigned G = gs(n * B) < 1024 ? gs(n * B) : 1024;
    hipLaunchKernelGGL(k_quad_loss, dim3(G), dim3(256), 0, st, yhat, gram, n, B, dy, partial);
    TBDG_HIP(hipGetLastError());
    return (int)G;
}

int net_mse(hipStream_t st, const float* yhat, const float* y, int64_t n, float* dy, double* partial) {
    const unsigned G = gs(n) < 1024 ? gs(n) : 1024;
    hipLaunchKernelGGL(k_mse, dim3(G), dim3(256), 0, st, yhat, y, n, dy, partial);
    TBDG_HIP(hipGetLastError());
    return (int)G;
}

void net_adam(hipStream_t st, int64_t n, float* theta, const float* g, float* m, float* v, float lr,
              float b1, float b2, float eps, float c1, float c2) {
    hipLaunchKernelGGL(k_adam, dim3(gs(n)), dim3(256), 0, st, n, theta, g, m, v, lr, b1, b2, eps, c1, c2);
    TBDG_HIP(hipGetLastError());
}

}  // namespace trbdg
