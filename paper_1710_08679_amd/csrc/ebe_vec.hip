// Nodal kernels of the multigrid preconditioner (Algorithm 1(a)): the
// quadratic <-> linear grid transfers P1 / P1^T and the 3x3 block-Jacobi
// application z = M^-1 e.  All vectors use the [node][component][case]
// layout; one work-item per stored value (transfers) or per (node, case)
// (block Jacobi), so consecutive lanes touch consecutive addresses.
#include <hip/hip_runtime.h>

#include "ebe_internal.h"

namespace ebe {
namespace {

constexpr int kBlock = 256;

inline unsigned grid_for(int64_t work) {
  int64_t g = (work + kBlock - 1) / kBlock;
  return unsigned(g < 1 ? 1 : g);
}

// y[N] = P1 x[Nv]: corners copied, edge node = mean of its two corners
template <typename T, bool BC>
__global__ __launch_bounds__(kBlock) void k_prolong(const int32_t* __restrict__ ends,
                                                    const uint8_t* __restrict__ fix,
                                                    const T* __restrict__ x, T* __restrict__ y,
                                                    int64_t n_nodes, int64_t n_vertices, int nrhs) {
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  const int64_t w = 3 * int64_t(nrhs);
  if (i >= n_nodes * w) return;
  const int64_t node = i / w;
  const int64_t rem = i - node * w;
  T v;
  if (node < n_vertices) {
    v = x[i];
  } else {
    const int64_t k = node - n_vertices;
    const int32_t p = ends[2 * k], q = ends[2 * k + 1];
    v = T(0.5) * (x[p * w + rem] + x[q * w + rem]);
  }
  if (BC && ((fix[node] >> (rem / nrhs)) & 1)) v = T(0);
  y[i] = v;
}

// y[Nv] = P1^T x[N]: corner value plus half of each incident edge-node value
template <typename T, bool BC>
__global__ __launch_bounds__(kBlock) void k_restrict(const int32_t* __restrict__ off,
                                                     const int32_t* __restrict__ idx,
                                                     const uint8_t* __restrict__ fix,
                                                     const T* __restrict__ x, T* __restrict__ y,
                                                     int64_t n_vertices, int nrhs) {
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  const int64_t w = 3 * int64_t(nrhs);
  if (i >= n_vertices * w) return;
  const int64_t v = i / w;
  const int64_t rem = i - v * w;
  T acc = T(0);
  for (int32_t k = off[v]; k < off[v + 1]; ++k) acc += x[int64_t(idx[k]) * w + rem];
  T out = x[i] + T(0.5) * acc;
  if (BC && ((fix[v] >> (rem / nrhs)) & 1)) out = T(0);
  y[i] = out;
}

// Level 2 (aggregates): y[Nv] = P2 x[Na] with the smoothed prolongator held
// by fine rows (width slots: aggregate id or -1, and a 3x3 block each); one
// work-item per fine value (row, component, case)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_prolong_p2(const int32_t* __restrict__ pcol, int width,
                                                       const T* __restrict__ pval, const T* __restrict__ x,
                                                       T* __restrict__ y, int64_t nv, int nrhs) {
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  const int64_t w3 = 3 * int64_t(nrhs);
  if (i >= nv * w3) return;
  const int64_t v = i / w3;
  const int64_t rem = i - v * w3;
  const int p = int(rem / nrhs);
  const int j = int(rem - int64_t(p) * nrhs);
  double acc = 0.0;
  for (int w = 0; w < width; ++w) {
    const int32_t J = pcol[v * width + w];
    if (J < 0) break;
    const T* b = pval + (v * width + w) * 9 + 3 * p;
    const T* xs = x + int64_t(J) * w3 + j;
    acc += double(b[0]) * double(xs[0]) + double(b[1]) * double(xs[nrhs]) + double(b[2]) * double(xs[2 * nrhs]);
  }
  y[i] = T(acc);
}

// y[Na] = P2^T x[Nv]: for aggregate I, the P2 entries naming it (fine rows in
// increasing order), each block transposed; zero at fixed coarse DOFs
template <typename T>
__global__ __launch_bounds__(kBlock) void k_restrict_p2(const int32_t* __restrict__ toff,
                                                        const int32_t* __restrict__ tidx, int width,
                                                        const T* __restrict__ pval, const uint8_t* __restrict__ cfix,
                                                        const T* __restrict__ x, T* __restrict__ y, int64_t na,
                                                        int nrhs) {
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  const int64_t w3 = 3 * int64_t(nrhs);
  if (i >= na * w3) return;
  const int64_t a = i / w3;
  const int64_t rem = i - a * w3;
  const int q = int(rem / nrhs);
  const int j = int(rem - int64_t(q) * nrhs);
  double acc = 0.0;
  if (!((cfix[a] >> q) & 1))
    for (int32_t t = toff[a]; t < toff[a + 1]; ++t) {
      const int64_t e = tidx[t];
      const int64_t v = e / width;
      const T* b = pval + e * 9 + q;
      const T* xs = x + v * w3 + j;
      acc += double(b[0]) * double(xs[0]) + double(b[3]) * double(xs[nrhs]) + double(b[6]) * double(xs[2 * nrhs]);
    }
  y[i] = T(acc);
}

// y = M^-1 x with symmetric inverse blocks (xx yy zz yz zx xy)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_bjacobi(const T* __restrict__ minv,
                                                    const T* __restrict__ x, T* __restrict__ y,
                                                    int64_t n, int nrhs) {
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= n * nrhs) return;
  const int64_t node = i / nrhs;
  const int r = int(i - node * nrhs);
  const T* m = minv + 6 * node;
  const int64_t b = node * 3 * nrhs + r;
  const T x0 = x[b], x1 = x[b + nrhs], x2 = x[b + 2 * nrhs];
  y[b] = m[0] * x0 + m[5] * x1 + m[4] * x2;
  y[b + nrhs] = m[5] * x0 + m[1] * x1 + m[3] * x2;
  y[b + 2 * nrhs] = m[4] * x0 + m[3] * x1 + m[2] * x2;
}

}  // namespace

hipError_t launch_prolong(const ebe_mesh* m, ebe_dtype dt, int nrhs, const void* x, void* y, bool bc,
                          hipStream_t s) {
  const unsigned g = grid_for(m->n_nodes * 3 * nrhs);
  const int32_t* ends = m->edge_ends.as<int32_t>();
  const uint8_t* fix = m->fix.as<uint8_t>();
  if (dt == EBE_F64) {
    if (bc)
      hipLaunchKernelGGL((k_prolong<double, true>), dim3(g), dim3(kBlock), 0, s, ends, fix,
                         static_cast<const double*>(x), static_cast<double*>(y), m->n_nodes, m->n_vertices, nrhs);
    else
      hipLaunchKernelGGL((k_prolong<double, false>), dim3(g), dim3(kBlock), 0, s, ends, fix,
                         static_cast<const double*>(x), static_cast<double*>(y), m->n_nodes, m->n_vertices, nrhs);
  } else {
    if (bc)
      hipLaunchKernelGGL((k_prolong<float, true>), dim3(g), dim3(kBlock), 0, s, ends, fix,
                         static_cast<const float*>(x), static_cast<float*>(y), m->n_nodes, m->n_vertices, nrhs);
    else
      hipLaunchKernelGGL((k_prolong<float, false>), dim3(g), dim3(kBlock), 0, s, ends, fix,
                         static_cast<const float*>(x), static_cast<float*>(y), m->n_nodes, m->n_vertices, nrhs);
  }
  return hipGetLastError();
}

hipError_t launch_restrict(const ebe_mesh* m, ebe_dtype dt, int nrhs, const void* x, void* y, bool bc,
                           hipStream_t s) {
  const unsigned g = grid_for(m->n_vertices * 3 * nrhs);
  const int32_t* off = m->v2e_off.as<int32_t>();
  const int32_t* idx = m->v2e_idx.as<int32_t>();
  const uint8_t* fix = m->fix.as<uint8_t>();
  if (dt == EBE_F64) {
    if (bc)
      hipLaunchKernelGGL((k_restrict<double, true>), dim3(g), dim3(kBlock), 0, s, off, idx, fix,
                         static_cast<const double*>(x), static_cast<double*>(y), m->n_vertices, nrhs);
    else
      hipLaunchKernelGGL((k_restrict<double, false>), dim3(g), dim3(kBlock), 0, s, off, idx, fix,
                         static_cast<const double*>(x), static_cast<double*>(y), m->n_vertices, nrhs);
  } else {
    if (bc)
      hipLaunchKernelGGL((k_restrict<float, true>), dim3(g), dim3(kBlock), 0, s, off, idx, fix,
                         static_cast<const float*>(x), static_cast<float*>(y), m->n_vertices, nrhs);
    else
      hipLaunchKernelGGL((k_restrict<float, false>), dim3(g), dim3(kBlock), 0, s, off, idx, fix,
                         static_cast<const float*>(x), static_cast<float*>(y), m->n_vertices, nrhs);
  }
  return hipGetLastError();
}

hipError_t launch_prolong_p2(const ebe_mesh* m, ebe_dtype dt, int nrhs, const void* x, void* y, hipStream_t s) {
  const unsigned g = grid_for(m->n_vertices * 3 * nrhs);
  if (dt == EBE_F64)
    hipLaunchKernelGGL(k_prolong_p2<double>, dim3(g), dim3(kBlock), 0, s, m->p2_col.as<int32_t>(), m->p2_width,
                       m->p2_val[0].as<double>(), static_cast<const double*>(x), static_cast<double*>(y),
                       m->n_vertices, nrhs);
  else
    hipLaunchKernelGGL(k_prolong_p2<float>, dim3(g), dim3(kBlock), 0, s, m->p2_col.as<int32_t>(), m->p2_width,
                       m->p2_val[1].as<float>(), static_cast<const float*>(x), static_cast<float*>(y), m->n_vertices,
                       nrhs);
  return hipGetLastError();
}

hipError_t launch_restrict_p2(const ebe_mesh* m, ebe_dtype dt, int nrhs, const void* x, void* y, hipStream_t s) {
  if (m->n_agg < 1) return hipSuccess;
  const unsigned g = grid_for(m->n_agg * 3 * nrhs);
  if (dt == EBE_F64)
    hipLaunchKernelGGL(k_restrict_p2<double>, dim3(g), dim3(kBlock), 0, s, m->p2t_off.as<int32_t>(),
                       m->p2t_idx.as<int32_t>(), m->p2_width, m->p2_val[0].as<double>(), m->cfix.as<uint8_t>(),
                       static_cast<const double*>(x), static_cast<double*>(y), m->n_agg, nrhs);
  else
    hipLaunchKernelGGL(k_restrict_p2<float>, dim3(g), dim3(kBlock), 0, s, m->p2t_off.as<int32_t>(),
                       m->p2t_idx.as<int32_t>(), m->p2_width, m->p2_val[1].as<float>(), m->cfix.as<uint8_t>(),
                       static_cast<const float*>(x), static_cast<float*>(y), m->n_agg, nrhs);
  return hipGetLastError();
}

hipError_t launch_bjacobi(const ebe_mesh* m, int level, ebe_dtype dt, int nrhs, const void* x, void* y,
                          hipStream_t s) {
  const int64_t n = level_rows(m, level);
  const unsigned g = grid_for(n * nrhs);
  if (dt == EBE_F64)
    hipLaunchKernelGGL(k_bjacobi<double>, dim3(g), dim3(kBlock), 0, s, m->minv64[level].as<double>(),
                       static_cast<const double*>(x), static_cast<double*>(y), n, nrhs);
  else
    hipLaunchKernelGGL(k_bjacobi<float>, dim3(g), dim3(kBlock), 0, s, m->minv32[level].as<float>(),
                       static_cast<const float*>(x), static_cast<float*>(y), n, nrhs);
  return hipGetLastError();
}

}  // namespace ebe
