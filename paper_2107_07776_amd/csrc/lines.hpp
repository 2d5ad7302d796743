// Index helpers of the line-structured operator kernels on affine
// Cartesian boxes (node layout inside a cell, neighbour cells, block maps).
#pragma once

#include "internal.hpp"

namespace trbdg {
namespace lines {

constexpr int ipow(int b, int e) { return e == 0 ? 1 : b * ipow(b, e - 1); }

template <int DIM, int N>
struct Lay {
    static constexpr int NB = ipow(N, DIM);
    static constexpr int CPB = (256 / NB) > 0 ? (256 / NB) : 1;
    static constexpr int THREADS = CPB * NB;
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
    __device__ static inline double wtan(const double* W, int t) {
        return DIM == 2 ? W[t] : W[t % N] * W[t / N];
    }
    __device__ static inline double wnode(const double* W, int nd) {
        double w = 1.0;
        for (int a = 0; a < DIM; ++a) w *= W[coord(nd, a)];
        return w;
    }
};

// q = r / n for 0 <= r < 2^31 from a double reciprocal, corrected to exact.
__device__ inline int div_fast(int r, int n, double inv_n) {
    int q = (int)((double)r * inv_n);
    if (q * n > r) --q;
    else if ((q + 1) * n <= r) ++q;
    return q;
}

// Cell coordinates and the two neighbours of a cell along every direction.
template <int DIM>
struct Nbrs {
    int left[3], right[3];
    __device__ Nbrs(const Geom& g, const LineGeom& lg, int cell) {
        int r = cell;
        int stride = 1;
        for (int a = 0; a < DIM; ++a) {
            const int n = g.nc[a];
            const int q = div_fast(r, n, lg.inv_nc[a]);
            const int ca = r - q * n;
            r = q;
            left[a] = ca > 0 ? cell - stride : (lg.periodic[a] ? cell + (n - 1) * stride : -1);
            right[a] = ca < n - 1 ? cell + stride : (lg.periodic[a] ? cell - (n - 1) * stride : -1);
            stride *= n;
        }
    }
};

// Blocks are always launched with 256 threads (four full waves, so the
// wave-level shuffles of the block reductions never read an inactive lane);
// threads beyond CPB whole cells idle in phases 1 and 3.
template <int DIM, int N>
struct FaceLay {
    static constexpr int NB = ipow(N, DIM);
    static constexpr int NF = ipow(N, DIM - 1);
    static constexpr int CPB = (256 / NB) > 0 ? (256 / NB) : 1;
    static constexpr int THREADS = 256;
};

__device__ inline int xcd_block(int b, int G) {
    const int x = b & 7, i = b >> 3;
    const int q = G >> 3, r = G & 7;
    return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// Cell of local slot lc in tile `blk` (tiles of cpb x-consecutive cells):
// with zc == 0 tiles are numbered x-fastest; otherwise z-fastest within
// chunks of zc z-planes (then x, then y, then chunk), so that the tiles
// holding a cell's z-neighbours run next to it and the neighbour values it
// gathers are still in L2 when their own tile reads them.  Needs
// nc[0] % cpb == 0 and nc[2] % zc == 0.  Returns -1 past the last cell.
__device__ inline int tile_cell(int blk, int lc, const Geom& g, int cpb, int zc, int Nc) {
    if (zc == 0) {
        const int c = blk * cpb + lc;
        return c < Nc ? c : -1;
    }
    const int ntx = g.nc[0] / cpb;
    int t = blk;
    const int zz = t % zc;
    t /= zc;
    const int tx = t % ntx;
    t /= ntx;
    const int ty = t % g.nc[1];
    const int tz = (t / g.nc[1]) * zc + zz;
    if (tz >= g.nc[2]) return -1;
    return (tx * cpb + lc) + g.nc[0] * (ty + g.nc[1] * tz);
}

// z-chunk depth for tile_cell on this mesh (0: plain x-fastest order)
inline int tile_zchunk(int dim, const int* nc, int cpb) {
    if (dim != 3 || nc[0] % cpb != 0) return 0;
    for (int z : {4, 2}) if (nc[2] % z == 0) return z;
    return 0;
}

}  // namespace lines
}  // namespace trbdg
