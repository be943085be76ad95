// Nodal kernels of the multigrid preconditioner (Algorithm 1(a)): the grid
// transfers P1 / P1^T (quadratic <-> linear) and P2 / P2^T (linear <->
// aggregates) and the 3x3 block-Jacobi application z = M^-1 e.  All vectors
// use the [node][component][case] layout; one work-item per vector of a node
// row (transfers) or per (node, case) (block Jacobi), so consecutive lanes
// touch consecutive addresses.
#include <hip/hip_runtime.h>

#include "ebe_internal.h"

namespace ebe {
namespace {

constexpr int kBlock = 256;

template <typename T, int VW>
struct alignas(sizeof(T) * VW) VecT {
  T v[VW];
};

inline unsigned grid_for(int64_t work) {
  int64_t g = (work + kBlock - 1) / kBlock;
  return unsigned(g < 1 ? 1 : g);
}

// The transfers take the case count as a template parameter: one work-item
// per VW consecutive values of a node row (VW values of one component, VW
// dividing n), so index arithmetic is by constants and accesses are vectors.
template <typename T, int NR>
constexpr int xfer_vec() {
  int v = 16 / int(sizeof(T));
  while (v > 1 && NR % v != 0) v /= 2;
  return v;
}

// y[N] = P1 x[Nv]: corners copied, edge node = mean of its two corners
template <typename T, int NR, bool BC>
__global__ __launch_bounds__(kBlock) void k_prolong(const int32_t* __restrict__ ends,
                                                    const uint8_t* __restrict__ fix,
                                                    const T* __restrict__ x, T* __restrict__ y,
                                                    int64_t n_nodes, int64_t n_vertices) {
  constexpr int VW = xfer_vec<T, NR>(), W = 3 * NR, PR = W / VW;
  using V = VecT<T, VW>;
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= n_nodes * PR) return;
  const int64_t node = i / PR;
  const int off = int(i - node * PR) * VW;
  V v;
  if (node < n_vertices) {
    v = *reinterpret_cast<const V*>(x + node * W + off);
  } else {
    const int64_t k = node - n_vertices;
    const V a = *reinterpret_cast<const V*>(x + int64_t(ends[2 * k]) * W + off);
    const V b = *reinterpret_cast<const V*>(x + int64_t(ends[2 * k + 1]) * W + off);
#pragma unroll
    for (int t = 0; t < VW; ++t) v.v[t] = T(0.5) * (a.v[t] + b.v[t]);
  }
  if (BC && ((fix[node] >> (off / NR)) & 1)) {
#pragma unroll
    for (int t = 0; t < VW; ++t) v.v[t] = T(0);
  }
  *reinterpret_cast<V*>(y + node * W + off) = v;
}

// y[Nv] = P1^T x[N]: corner value plus half of each incident edge-node value
template <typename T, int NR, bool BC>
__global__ __launch_bounds__(kBlock) void k_restrict(const int32_t* __restrict__ eoff,
                                                     const int32_t* __restrict__ idx,
                                                     const uint8_t* __restrict__ fix,
                                                     const T* __restrict__ x, T* __restrict__ y,
                                                     int64_t n_vertices) {
  constexpr int VW = xfer_vec<T, NR>(), W = 3 * NR, PR = W / VW;
  using V = VecT<T, VW>;
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= n_vertices * PR) return;
  const int64_t v = i / PR;
  const int off = int(i - v * PR) * VW;
  T acc[VW];
#pragma unroll
  for (int t = 0; t < VW; ++t) acc[t] = T(0);
  for (int32_t k = eoff[v]; k < eoff[v + 1]; ++k) {
    const V e = *reinterpret_cast<const V*>(x + int64_t(idx[k]) * W + off);
#pragma unroll
    for (int t = 0; t < VW; ++t) acc[t] += e.v[t];
  }
  const V own = *reinterpret_cast<const V*>(x + v * W + off);
  V out;
  const bool fixed = BC && ((fix[v] >> (off / NR)) & 1);
#pragma unroll
  for (int t = 0; t < VW; ++t) out.v[t] = fixed ? T(0) : own.v[t] + T(0.5) * acc[t];
  *reinterpret_cast<V*>(y + v * W + off) = out;
}

// Level 2 (aggregates): y[Nv] = P2 x[Na] with the smoothed prolongator held
// by fine rows (width slots: aggregate id or -1, and a 3x3 block each)
template <typename T, int NR>
__global__ __launch_bounds__(kBlock) void k_prolong_p2(const int32_t* __restrict__ pcol, int width,
                                                       const T* __restrict__ pval, const T* __restrict__ x,
                                                       T* __restrict__ y, int64_t nv) {
  constexpr int VW = xfer_vec<T, NR>(), W = 3 * NR, PR = W / VW;
  using V = VecT<T, VW>;
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= nv * PR) return;
  const int64_t v = i / PR;
  const int off = int(i - v * PR) * VW;
  const int p = off / NR, j = off - p * NR;
  double acc[VW];
#pragma unroll
  for (int t = 0; t < VW; ++t) acc[t] = 0.0;
  for (int w = 0; w < width; ++w) {
    const int32_t J = pcol[v * width + w];
    if (J < 0) break;
    const T* b = pval + (v * width + w) * 9 + 3 * p;
    const T* xs = x + int64_t(J) * W + j;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const V xv = *reinterpret_cast<const V*>(xs + q * NR);
      const double bq = double(b[q]);
#pragma unroll
      for (int t = 0; t < VW; ++t) acc[t] += bq * double(xv.v[t]);
    }
  }
  V out;
#pragma unroll
  for (int t = 0; t < VW; ++t) out.v[t] = T(acc[t]);
  *reinterpret_cast<V*>(y + v * W + off) = out;
}

// y[Na] = P2^T x[Nv]: for aggregate I, the P2 entries naming it (fine rows in
// increasing order), each block transposed; zero at fixed coarse DOFs
template <typename T, int NR>
__global__ __launch_bounds__(kBlock) void k_restrict_p2(const int32_t* __restrict__ toff,
                                                        const int32_t* __restrict__ tidx, int width,
                                                        const T* __restrict__ pval, const uint8_t* __restrict__ cfix,
                                                        const T* __restrict__ x, T* __restrict__ y, int64_t na) {
  constexpr int VW = xfer_vec<T, NR>(), W = 3 * NR, PR = W / VW;
  using V = VecT<T, VW>;
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= na * PR) return;
  const int64_t a = i / PR;
  const int off = int(i - a * PR) * VW;
  const int q = off / NR, j = off - q * NR;
  double acc[VW];
#pragma unroll
  for (int t = 0; t < VW; ++t) acc[t] = 0.0;
  if (!((cfix[a] >> q) & 1))
    for (int32_t k = toff[a]; k < toff[a + 1]; ++k) {
      const int64_t e = tidx[k];
      const int64_t v = e / width;
      const T* b = pval + e * 9 + q;
      const T* xs = x + v * W + j;
#pragma unroll
      for (int p = 0; p < 3; ++p) {
        const V xv = *reinterpret_cast<const V*>(xs + p * NR);
        const double bp = double(b[3 * p]);
#pragma unroll
        for (int t = 0; t < VW; ++t) acc[t] += bp * double(xv.v[t]);
      }
    }
  V out;
#pragma unroll
  for (int t = 0; t < VW; ++t) out.v[t] = T(acc[t]);
  *reinterpret_cast<V*>(y + a * W + off) = out;
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

namespace {

template <typename T, int NR>
hipError_t xfer_p(int which, const ebe_mesh* m, const void* x, void* y, bool bc, hipStream_t s) {
  constexpr int PR = 3 * NR / xfer_vec<T, NR>();
  const T* xs = static_cast<const T*>(x);
  T* yd = static_cast<T*>(y);
  const int k = sizeof(T) == 8 ? 0 : 1;
  switch (which) {
    case 0:  // P1
      if (bc)
        hipLaunchKernelGGL((k_prolong<T, NR, true>), dim3(grid_for(m->n_nodes * PR)), dim3(kBlock), 0, s,
                           m->edge_ends.as<int32_t>(), m->fix.as<uint8_t>(), xs, yd, m->n_nodes, m->n_vertices);
      else
        hipLaunchKernelGGL((k_prolong<T, NR, false>), dim3(grid_for(m->n_nodes * PR)), dim3(kBlock), 0, s,
                           m->edge_ends.as<int32_t>(), m->fix.as<uint8_t>(), xs, yd, m->n_nodes, m->n_vertices);
      break;
    case 1:  // P1^T
      if (bc)
        hipLaunchKernelGGL((k_restrict<T, NR, true>), dim3(grid_for(m->n_vertices * PR)), dim3(kBlock), 0, s,
                           m->v2e_off.as<int32_t>(), m->v2e_idx.as<int32_t>(), m->fix.as<uint8_t>(), xs, yd,
                           m->n_vertices);
      else
        hipLaunchKernelGGL((k_restrict<T, NR, false>), dim3(grid_for(m->n_vertices * PR)), dim3(kBlock), 0, s,
                           m->v2e_off.as<int32_t>(), m->v2e_idx.as<int32_t>(), m->fix.as<uint8_t>(), xs, yd,
                           m->n_vertices);
      break;
    case 2:  // P2
      hipLaunchKernelGGL((k_prolong_p2<T, NR>), dim3(grid_for(m->n_vertices * PR)), dim3(kBlock), 0, s,
                         m->p2_col.as<int32_t>(), m->p2_width, m->p2_val[k].as<T>(), xs, yd, m->n_vertices);
      break;
    default:  // P2^T
      if (m->n_agg < 1) return hipSuccess;
      hipLaunchKernelGGL((k_restrict_p2<T, NR>), dim3(grid_for(m->n_agg * PR)), dim3(kBlock), 0, s,
                         m->p2t_off.as<int32_t>(), m->p2t_idx.as<int32_t>(), m->p2_width, m->p2_val[k].as<T>(),
                         m->cfix.as<uint8_t>(), xs, yd, m->n_agg);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t xfer(int which, const ebe_mesh* m, int nrhs, const void* x, void* y, bool bc, hipStream_t s) {
  switch (nrhs) {
#define EBE_CASE(n) \
  case n: return xfer_p<T, n>(which, m, x, y, bc, s);
    EBE_CASE(1) EBE_CASE(2) EBE_CASE(3) EBE_CASE(4) EBE_CASE(5) EBE_CASE(6) EBE_CASE(7) EBE_CASE(8)
    EBE_CASE(9) EBE_CASE(10) EBE_CASE(11) EBE_CASE(12) EBE_CASE(13) EBE_CASE(14) EBE_CASE(15) EBE_CASE(16)
#undef EBE_CASE
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_prolong(const ebe_mesh* m, ebe_dtype dt, int nrhs, const void* x, void* y, bool bc,
                          hipStream_t s) {
  return dt == EBE_F64 ? xfer<double>(0, m, nrhs, x, y, bc, s) : xfer<float>(0, m, nrhs, x, y, bc, s);
}

hipError_t launch_restrict(const ebe_mesh* m, ebe_dtype dt, int nrhs, const void* x, void* y, bool bc,
                           hipStream_t s) {
  return dt == EBE_F64 ? xfer<double>(1, m, nrhs, x, y, bc, s) : xfer<float>(1, m, nrhs, x, y, bc, s);
}

hipError_t launch_prolong_p2(const ebe_mesh* m, ebe_dtype dt, int nrhs, const void* x, void* y, hipStream_t s) {
  return dt == EBE_F64 ? xfer<double>(2, m, nrhs, x, y, false, s) : xfer<float>(2, m, nrhs, x, y, false, s);
}

hipError_t launch_restrict_p2(const ebe_mesh* m, ebe_dtype dt, int nrhs, const void* x, void* y, hipStream_t s) {
  return dt == EBE_F64 ? xfer<double>(3, m, nrhs, x, y, false, s) : xfer<float>(3, m, nrhs, x, y, false, s);
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
