// Kernels of the merged batch solves (batch.cpp): moving one member mesh's
// cases into and out of a merged (block-diagonal) system, and the per-case
// norms the merge needs.
//
// A merged system holds several small meshes side by side: member i's node v
// is merged node map_i[v], its cases are the merged system's first n_i cases
// (the others are zero for its nodes).  Each case is scaled to unit norm on
// the way in, so the merged solve's stopping test (the largest relative
// residual over cases) bounds every member's own relative residual.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "batch_kernels.h"

namespace ebe {
namespace {

constexpr int kB = 256;

// F[map[v]][c][r] = f[v][c][r] * scale[r] for r < n (F has nr cases)
__global__ __launch_bounds__(kB) void k_scatter_cases(const double* __restrict__ f, const int32_t* __restrict__ map,
                                                      int64_t N, int32_t n, const double* __restrict__ scale,
                                                      double* __restrict__ F, int32_t nr) {
  const int64_t w = int64_t(blockIdx.x) * kB + threadIdx.x;
  if (w >= N * 3 * n) return;
  const int64_t row = w / n;
  const int r = int(w - row * n);
  const int64_t v = row / 3;
  const int c = int(row - v * 3);
  F[(int64_t(map[v]) * 3 + c) * nr + r] = f[w] * scale[r];
}

// u[v][c][r] = U[map[v]][c][r] / scale[r] (0 where the case is zero)
__global__ __launch_bounds__(kB) void k_gather_cases(const double* __restrict__ U, const int32_t* __restrict__ map,
                                                     int64_t N, int32_t n, const double* __restrict__ scale,
                                                     double* __restrict__ u, int32_t nr) {
  const int64_t w = int64_t(blockIdx.x) * kB + threadIdx.x;
  if (w >= N * 3 * n) return;
  const int64_t row = w / n;
  const int r = int(w - row * n);
  const int64_t v = row / 3;
  const int c = int(row - v * 3);
  const double sc = scale[r];
  u[w] = sc > 0.0 ? U[(int64_t(map[v]) * 3 + c) * nr + r] / sc : 0.0;
}

// out[r] += sum over free DOFs of a[.][.][r]^2, and (b != null) out[n + r] +=
// sum over free DOFs of (a - b)^2; fix: bit c = DOF c fixed
__global__ __launch_bounds__(kB) void k_case_norms(const double* __restrict__ a, const double* __restrict__ b,
                                                   const uint8_t* __restrict__ fix, int64_t N, int32_t n,
                                                   double* __restrict__ out) {
  __shared__ double acc[2 * EBE_MAX_RHS];
  for (int i = threadIdx.x; i < 2 * EBE_MAX_RHS; i += kB) acc[i] = 0.0;
  __syncthreads();
  const int64_t total = N * 3 * n;
  for (int64_t w = int64_t(blockIdx.x) * kB + threadIdx.x; w < total; w += int64_t(gridDim.x) * kB) {
    const int64_t row = w / n;
    const int r = int(w - row * n);
    const int64_t v = row / 3;
    const int c = int(row - v * 3);
    if ((fix[v] >> c) & 1) continue;
    const double x = a[w];
    atomicAdd(&acc[r], x * x);
    if (b) {
      const double d = x - b[w];
      atomicAdd(&acc[EBE_MAX_RHS + r], d * d);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += kB) {
    unsafeAtomicAdd(out + i, acc[i]);
    if (b) unsafeAtomicAdd(out + n + i, acc[EBE_MAX_RHS + i]);
  }
}

unsigned grid_of(int64_t work) { return unsigned((work + kB - 1) / kB); }

}  // namespace

hipError_t launch_scatter_cases(const double* f, const int32_t* map, int64_t N, int32_t n, const double* scale,
                                double* F, int32_t nr, hipStream_t s) {
  if (N * n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_scatter_cases, dim3(grid_of(N * 3 * n)), dim3(kB), 0, s, f, map, N, n, scale, F, nr);
  return hipGetLastError();
}

hipError_t launch_gather_cases(const double* U, const int32_t* map, int64_t N, int32_t n, const double* scale,
                               double* u, int32_t nr, hipStream_t s) {
  if (N * n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_cases, dim3(grid_of(N * 3 * n)), dim3(kB), 0, s, U, map, N, n, scale, u, nr);
  return hipGetLastError();
}

hipError_t launch_case_norms(const double* a, const double* b, const uint8_t* fix, int64_t N, int32_t n, double* out,
                             hipStream_t s) {
  hipError_t e = launch_fill_zero(out, size_t(2) * n * sizeof(double), s);
  if (e != hipSuccess || N == 0) return e;
  const unsigned g = std::min<unsigned>(grid_of(N * 3 * n), 2048u);
  hipLaunchKernelGGL(k_case_norms, dim3(g), dim3(kB), 0, s, a, b, fix, N, n, out);
  return hipGetLastError();
}

}  // namespace ebe
