// Krylov reductions on a plain stream, for solvers that do not own a box
// context (the adaptive-mesh GMRES).  The kernels are the box solver's
// (blas.hip) with unscaled basis vectors.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace trbdg {

// out[j] = V_j . w for j < k and out[k] = w . w (V_j = V + j ldv); part holds
// (k + 1) G block partials, G blocks per vector (G <= 4096)
void kr_dots(hipStream_t st, int64_t n, int k, const double* V, int64_t ldv, const double* w,
             double* part, int G, double* out);
// w -= sum_{j<k} h_j V_j (h on the device, k <= 64), then *nn = |w|^2 and
// *inv = 1 / |w| (1 when w = 0); part holds G block partials
void kr_update_norm(hipStream_t st, int64_t n, int k, const double* V, int64_t ldv, const double* h,
                    double* w, double* part, int G, double* nn, double* inv);

}  // namespace trbdg
