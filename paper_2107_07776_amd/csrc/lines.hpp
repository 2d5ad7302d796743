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

}  // namespace lines
}  // namespace trbdg
