// Launchers of the merged batch solves' kernels (batch_kernels.hip).
#pragma once

#include "ebe_internal.h"

namespace ebe {

// F[map[v]][c][r] = f[v][c][r] * scale[r], r < n (F: [.][3][nr]; its other entries untouched)
hipError_t launch_scatter_cases(const double* f, const int32_t* map, int64_t N, int32_t n, const double* scale,
                                double* F, int32_t nr, hipStream_t s);
// u[v][c][r] = U[map[v]][c][r] / scale[r] (0 where scale[r] = 0), r < n
hipError_t launch_gather_cases(const double* U, const int32_t* map, int64_t N, int32_t n, const double* scale,
                               double* u, int32_t nr, hipStream_t s);
// out[r] = sum over free DOFs of a_r^2; out[n + r] = sum over free DOFs of
// (a_r - b_r)^2 when b is given (out: device, 2 n doubles, overwritten)
hipError_t launch_case_norms(const double* a, const double* b, const uint8_t* fix, int64_t N, int32_t n, double* out,
                             hipStream_t s);

}  // namespace ebe
