// Adjoint element kernel: g_e = - sum_c lambda_{c,e}^T (K_e / E_e) u_{c,e}.
//
// K_e is linear in E_e at fixed Poisson ratio, so dK_e/dE_e is the element
// operator rebuilt with (lambda/E, mu/E).  Each element forms that operator on
// the fly (as the EBE product does, Section 2) for every case, contracts it
// with the adjoint state and writes its own entry: no scatter, no atomics.
// One work-item per (element, case); the cases of an element are adjacent
// lanes and are summed with a cross-lane reduction.
#include <hip/hip_runtime.h>

#include "ebe_internal.h"
#include "p2_element.h"

namespace ebe {
namespace {

constexpr int kBlock = 256;

template <typename T> struct Pair;
template <> struct Pair<double> { using type = double2; };
template <> struct Pair<float> { using type = float2; };

template <typename T, int NR>
__global__ __launch_bounds__(kBlock) void k_adjoint(const int32_t* __restrict__ conn,
                                                    const double4* __restrict__ xv,
                                                    const double* __restrict__ young,
                                                    const typename Pair<T>::type* __restrict__ lame,
                                                    const T* __restrict__ u, const T* __restrict__ lam,
                                                    T* __restrict__ g, int64_t nelem) {
  // NR is a power of two <= 16 so that an element's cases never straddle a wavefront.
  const int64_t t = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  const int64_t e = t / NR;
  const int r = int(t - e * NR);
  const bool live = e < nelem;
  T acc = T(0);
  if (live) {
    int32_t cw[10];
#pragma unroll
    for (int a = 0; a < 10; ++a) cw[a] = conn[e * 10 + a];
    T G[4][3];
    const T V = tet_geometry<T>(xv[cw[0] & kIdxMask], xv[cw[1] & kIdxMask], xv[cw[2] & kIdxMask],
                                xv[cw[3] & kIdxMask], G);
    const auto lm = lame[e];
    const T s = V * T(0.05) / T(young[e]);
    // streaming element operator: nodal values read as needed, each nodal
    // force contracted with the adjoint state as soon as it is known
    T unused = T(0);
    p2_apply<T>(
        G, T(lm.x) * s, T(lm.y) * s,
        [&](int a, int c) -> T {
          return ((cw[a] >> (kIdxBits + c)) & 1) ? T(0) : u[size_t(cw[a] & kIdxMask) * (3 * NR) + c * NR + r];
        },
        [&](int a, const T f[3]) {
          const T* p = lam + size_t(cw[a] & kIdxMask) * (3 * NR) + r;
#pragma unroll
          for (int c = 0; c < 3; ++c)
            if (!((cw[a] >> (kIdxBits + c)) & 1)) acc += p[c * NR] * f[c];
        },
        false, unused);
  }
#pragma unroll
  for (int off = 1; off < NR; off <<= 1) acc += __shfl_xor(acc, off, NR);
  if (live && r == 0) g[e] = -acc;
}

// general nrhs: loop over cases in one work-item
template <typename T>
__global__ __launch_bounds__(kBlock) void k_adjoint_loop(const int32_t* __restrict__ conn,
                                                         const double4* __restrict__ xv,
                                                         const double* __restrict__ young,
                                                         const typename Pair<T>::type* __restrict__ lame,
                                                         const T* __restrict__ u, const T* __restrict__ lam,
                                                         T* __restrict__ g, int64_t nelem, int nrhs) {
  const int64_t e = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (e >= nelem) return;
  int32_t cw[10];
#pragma unroll
  for (int a = 0; a < 10; ++a) cw[a] = conn[e * 10 + a];
  T G[4][3];
  const T V = tet_geometry<T>(xv[cw[0] & kIdxMask], xv[cw[1] & kIdxMask], xv[cw[2] & kIdxMask],
                              xv[cw[3] & kIdxMask], G);
  const auto lm = lame[e];
  const T s = V * T(0.05) / T(young[e]);
  T acc = T(0);
  for (int r = 0; r < nrhs; ++r) {
    T unused = T(0);
    p2_apply<T>(
        G, T(lm.x) * s, T(lm.y) * s,
        [&](int a, int c) -> T {
          return ((cw[a] >> (kIdxBits + c)) & 1) ? T(0) : u[size_t(cw[a] & kIdxMask) * 3 * nrhs + c * nrhs + r];
        },
        [&](int a, const T f[3]) {
          const T* p = lam + size_t(cw[a] & kIdxMask) * 3 * nrhs + r;
#pragma unroll
          for (int c = 0; c < 3; ++c)
            if (!((cw[a] >> (kIdxBits + c)) & 1)) acc += p[c * nrhs] * f[c];
        },
        false, unused);
  }
  g[e] = -acc;
}

template <typename T>
hipError_t adjoint_t(const ebe_mesh* m, int nrhs, const void* u, const void* lam, void* g, hipStream_t s) {
  using P = typename Pair<T>::type;
  const P* lame = (sizeof(T) == 8) ? reinterpret_cast<const P*>(m->lame64.as<void>())
                                   : reinterpret_cast<const P*>(m->lame32.as<void>());
  const T* uu = static_cast<const T*>(u);
  const T* ll = static_cast<const T*>(lam);
  T* gg = static_cast<T*>(g);
  auto grid = [&](int64_t w) { return dim3(unsigned((w + kBlock - 1) / kBlock)); };
  switch (nrhs) {
#define EBE_ADJ(n)                                                                                    \
  case n:                                                                                             \
    hipLaunchKernelGGL((k_adjoint<T, n>), grid(m->n_elem * n), dim3(kBlock), 0, s, m->conn.as<int32_t>(), \
                       m->xv.as<double4>(), m->young.as<double>(), lame, uu, ll, gg, m->n_elem);      \
    break;
    EBE_ADJ(1) EBE_ADJ(2) EBE_ADJ(4) EBE_ADJ(8) EBE_ADJ(16)
#undef EBE_ADJ
    default:
      hipLaunchKernelGGL(k_adjoint_loop<T>, grid(m->n_elem), dim3(kBlock), 0, s, m->conn.as<int32_t>(),
                         m->xv.as<double4>(), m->young.as<double>(), lame, uu, ll, gg, m->n_elem, nrhs);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_adjoint(const ebe_mesh* m, ebe_dtype dt, int nrhs, const void* u, const void* lam,
                          void* g, hipStream_t s) {
  return dt == EBE_F64 ? adjoint_t<double>(m, nrhs, u, lam, g, s) : adjoint_t<float>(m, nrhs, u, lam, g, s);
}

}  // namespace ebe
