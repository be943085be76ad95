// Kernels of the Green's-function pipeline (Section 5, Eq. (4)-(5); the
// split-node fault loading of Section 2):
//   k_split_forces   f_c = sum over the elements touching the fault of
//                    -(side_e / 2) K_e s_{c,e}, where the slip s_c of basis
//                    function c is its value at the fault nodes times its
//                    slip direction (a fault node carries two displacements
//                    whose difference is the slip; the mean field v then
//                    solves K v = f on the ordinary mesh);
//   k_gather_obs     G[3 s + d][col] = u(station s, component d, case);
//   k_lsq_qr         for one regularisation weight alpha, the least-squares
//                    solution of the stacked system [G; alpha L] a = [d; 0]
//                    of Eq. (5) by Householder QR, and the residual norm
//                    ||G a - d|| and seminorm ||L a|| (the L-curve point);
//   k_lcurve_corner  curvature of (log rho, log eta) as a function of
//                    log alpha and its maximum (Hansen's L-curve corner).
#include <hip/hip_runtime.h>

#include <cmath>

#include "ebe_internal.h"
#include "greens.h"
#include "p2_element.h"

namespace ebe {
namespace {

// One work-item per (fault element, case).  Element geometry from the corner
// coordinates and (lambda, mu), as the products form it; forces added to f
// with FP64 atomics (few elements touch the fault).
template <int NR>
__global__ __launch_bounds__(256) void k_split_forces(const int32_t* __restrict__ conn,
                                                      const double4* __restrict__ xv,
                                                      const double2* __restrict__ lame,
                                                      const int32_t* __restrict__ fel,
                                                      const int8_t* __restrict__ fside,
                                                      const int32_t* __restrict__ frow,
                                                      const double* __restrict__ basis,
                                                      const double* __restrict__ dirs, int32_t nbasis,
                                                      int32_t col0, int32_t nfel, double* __restrict__ f) {
  const int64_t w = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (w >= int64_t(nfel) * NR) return;
  const int k = int(w / NR), r = int(w - int64_t(k) * NR);
  const int64_t e = fel[k];
  const int32_t* ce = conn + e * 10;
  double G[4][3];
  const double V = tet_geometry<double>(xv[ce[0] & kIdxMask], xv[ce[1] & kIdxMask], xv[ce[2] & kIdxMask],
                                        xv[ce[3] & kIdxMask], G);
  const double2 lm = lame[e];
  const double s20 = V * 0.05;
  // slip of this case at the element's nodes (zero off the fault)
  const int col = col0 + r;
  const double dx = dirs[col * 3 + 0], dy = dirs[col * 3 + 1], dz = dirs[col * 3 + 2];
  double s[10][3];
#pragma unroll
  for (int a = 0; a < 10; ++a) {
    const int32_t fr = frow[int64_t(k) * 10 + a];
    const double b = fr >= 0 ? basis[int64_t(fr) * nbasis + col] : 0.0;
    s[a][0] = b * dx;
    s[a][1] = b * dy;
    s[a][2] = b * dz;
  }
  double fe[10][3];
  p2_forces<double>(G, lm.x * s20, lm.y * s20, s, fe);
  const double wgt = -0.5 * double(fside[k]);
#pragma unroll
  for (int a = 0; a < 10; ++a) {
    const int64_t row = int64_t(ce[a] & kIdxMask) * 3 * NR + r;
#pragma unroll
    for (int c = 0; c < 3; ++c) unsafeAtomicAdd(f + row + c * NR, wgt * fe[a][c]);
  }
}

// G[3 s + d][col0 + r] = u[st[s]][d][r]
__global__ __launch_bounds__(256) void k_gather_obs(const double* __restrict__ u, int32_t nrhs,
                                                    const int32_t* __restrict__ st, int32_t nst,
                                                    double* __restrict__ G, int32_t ld, int32_t col0) {
  const int64_t w = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (w >= int64_t(nst) * 3 * nrhs) return;
  const int64_t row = w / nrhs;
  const int r = int(w - row * nrhs);
  const int32_t s = int32_t(row / 3), d = int32_t(row - int64_t(s) * 3);
  G[row * ld + col0 + r] = u[(int64_t(st[s]) * 3 + d) * nrhs + r];
}

constexpr int kQrThreads = 256;

// block-wide sum of one value per work-item (all work-items get the sum)
__device__ double block_sum(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wv] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int i = 0; i < kQrThreads / 64; ++i) t += red[i];
  return t;
}

// One workgroup per alpha.  The stacked matrix A = [G; alpha L] (m x nb,
// m = nobs + nreg) is copied column-major into this workgroup's workspace
// with b = [d; 0] as column nb, then reduced to R by Householder
// reflections (one wavefront per column when a reflection is applied), and
// R a = Q^T b is solved by back substitution.  A must have full column rank
// (alpha > 0 and L of full rank guarantee it).
__global__ __launch_bounds__(kQrThreads) void k_lsq_qr(const double* __restrict__ Gm, const double* __restrict__ d,
                                                       const double* __restrict__ L, const double* __restrict__ alphas,
                                                       int32_t nobs, int32_t nreg, int32_t nb,
                                                       double* __restrict__ work, double* __restrict__ a_out,
                                                       double* __restrict__ rho, double* __restrict__ eta) {
  __shared__ double red[kQrThreads / 64];
  __shared__ double coef[kLsqMaxBasis];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  constexpr int NW = kQrThreads / 64;
  const int ia = blockIdx.x;
  const double al = alphas[ia];
  const int m = nobs + nreg;
  double* A = work + int64_t(ia) * int64_t(m) * (nb + 1);  // column j at A + j * m
  for (int64_t i = tid; i < int64_t(m) * (nb + 1); i += kQrThreads) {
    const int j = int(i / m), row = int(i - int64_t(j) * m);
    double v;
    if (j < nb) v = row < nobs ? Gm[int64_t(row) * nb + j] : al * L[int64_t(row - nobs) * nb + j];
    else v = row < nobs ? d[row] : 0.0;
    A[i] = v;
  }
  __syncthreads();
  for (int k = 0; k < nb; ++k) {
    double* ak = A + int64_t(k) * m;
    double ss = 0.0;
    for (int i = k + tid; i < m; i += kQrThreads) ss += ak[i] * ak[i];
    const double sigma = sqrt(block_sum(ss, red));
    const double x0 = ak[k];
    const double beta = x0 >= 0.0 ? -sigma : sigma;  // R[k][k]; the sign avoids cancellation in v_k
    const double v0 = x0 - beta;                     // v = a_k - beta e_k (below the diagonal: a_k itself)
    __syncthreads();
    if (sigma > 0.0) {
      // apply H_k = I - 2 v v^T / (v^T v) to the columns j > k (and b);
      // v^T v = -2 beta v_k, so a_j += v (v^T a_j) / (beta v_k)
      const double scale = -1.0 / (v0 * beta);
      for (int j = k + 1 + wv; j <= nb; j += NW) {
        double* aj = A + int64_t(j) * m;
        double dot = lane == 0 ? v0 * aj[k] : 0.0;
        for (int i = k + 1 + lane; i < m; i += 64) dot += ak[i] * aj[i];
        for (int off = 32; off > 0; off >>= 1) dot += __shfl_xor(dot, off, 64);
        const double t = dot * scale;
        if (lane == 0) aj[k] -= t * v0;
        for (int i = k + 1 + lane; i < m; i += 64) aj[i] -= t * ak[i];
      }
    }
    __syncthreads();
    if (tid == 0) ak[k] = beta;  // R[k][k]; below the diagonal of column k is no longer needed
    __syncthreads();
  }
  // back substitution R a = (Q^T b)[0:nb], R[i][j] = A[j * m + i]
  const double* qb = A + int64_t(nb) * m;
  for (int i = nb - 1; i >= 0; --i) {
    double s = 0.0;
    for (int j = i + 1 + tid; j < nb; j += kQrThreads) s += A[int64_t(j) * m + i] * coef[j];
    s = block_sum(s, red);
    if (tid == 0) coef[i] = (qb[i] - s) / A[int64_t(i) * m + i];
    __syncthreads();
  }
  for (int j = tid; j < nb; j += kQrThreads) a_out[int64_t(ia) * nb + j] = coef[j];
  // rho = ||G a - d||, eta = ||L a||, from G, L and d themselves
  double rr = 0.0, ee = 0.0;
  for (int i = tid; i < nobs; i += kQrThreads) {
    double t = -d[i];
    for (int j = 0; j < nb; ++j) t += Gm[int64_t(i) * nb + j] * coef[j];
    rr += t * t;
  }
  for (int i = tid; i < nreg; i += kQrThreads) {
    double t = 0.0;
    for (int j = 0; j < nb; ++j) t += L[int64_t(i) * nb + j] * coef[j];
    ee += t * t;
  }
  rr = block_sum(rr, red);
  ee = block_sum(ee, red);
  if (tid == 0) {
    rho[ia] = sqrt(rr);
    eta[ia] = sqrt(ee);
  }
}

// first derivative of samples f(t_i) on a nonuniform grid: second-order
// central differences inside (the three-point formula exact for quadratics),
// one-sided first-order differences at the two ends
__device__ double diff1(const double* f, const double* t, int i, int n) {
  if (i == 0) return (f[1] - f[0]) / (t[1] - t[0]);
  if (i == n - 1) return (f[n - 1] - f[n - 2]) / (t[n - 1] - t[n - 2]);
  const double hs = t[i] - t[i - 1], hd = t[i + 1] - t[i];
  return (hs * hs * f[i + 1] + (hd * hd - hs * hs) * f[i] - hd * hd * f[i - 1]) / (hs * hd * (hd + hs));
}

// One workgroup: curvature of the curve (log rho, log eta) parametrised by
// log alpha at every alpha, and the index of its largest value (the first
// one, if several are equal).  Needs n_alpha >= 3 and n_alpha <= kLcurveMax.
__global__ __launch_bounds__(256) void k_lcurve_corner(const double* __restrict__ alphas,
                                                       const double* __restrict__ rho,
                                                       const double* __restrict__ eta, int32_t n,
                                                       double* __restrict__ curv, int32_t* __restrict__ corner) {
  __shared__ double t[kLcurveMax], x[kLcurveMax], y[kLcurveMax], dx[kLcurveMax], dy[kLcurveMax];
  __shared__ double kap[kLcurveMax];
  for (int i = threadIdx.x; i < n; i += 256) {
    t[i] = log(alphas[i]);
    x[i] = log(rho[i]);
    y[i] = log(eta[i]);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += 256) {
    dx[i] = diff1(x, t, i, n);
    dy[i] = diff1(y, t, i, n);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += 256) {
    const double ddx = diff1(dx, t, i, n), ddy = diff1(dy, t, i, n);
    const double sp = dx[i] * dx[i] + dy[i] * dy[i];
    kap[i] = (dx[i] * ddy - ddx * dy[i]) / (sp * sqrt(sp));
    curv[i] = kap[i];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int best = 0;
    for (int i = 1; i < n; ++i)
      if (kap[i] > kap[best]) best = i;
    *corner = best;
  }
}

}  // namespace

hipError_t launch_split_forces(const ebe_mesh* m, const int32_t* fel, const int8_t* fside, const int32_t* frow,
                               const double* basis, const double* dirs, int32_t nbasis, int32_t nfel, int32_t col0,
                               int32_t nrhs, double* f, hipStream_t s) {
  hipError_t e = launch_fill_zero(f, size_t(m->n_nodes) * 3 * nrhs * sizeof(double), s);
  if (e != hipSuccess || nfel == 0) return e;
  const int64_t work = int64_t(nfel) * nrhs;
  const dim3 grid(unsigned((work + 255) / 256));
  switch (nrhs) {
#define EBE_CASE(n)                                                                                             \
  case n:                                                                                                       \
    hipLaunchKernelGGL((k_split_forces<n>), grid, dim3(256), 0, s, m->conn.as<int32_t>(), m->xv.as<double4>(), \
                       m->lame64.as<double2>(), fel, fside, frow, basis, dirs, nbasis, col0, nfel, f);          \
    break;
    EBE_CASE(1) EBE_CASE(2) EBE_CASE(3) EBE_CASE(4) EBE_CASE(5) EBE_CASE(6) EBE_CASE(7) EBE_CASE(8)
    EBE_CASE(9) EBE_CASE(10) EBE_CASE(11) EBE_CASE(12) EBE_CASE(13) EBE_CASE(14) EBE_CASE(15) EBE_CASE(16)
#undef EBE_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_gather_obs(const double* u, int32_t nrhs, const int32_t* st, int32_t nst, double* G, int32_t ld,
                             int32_t col0, hipStream_t s) {
  const int64_t work = int64_t(nst) * 3 * nrhs;
  if (work == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_obs, dim3(unsigned((work + 255) / 256)), dim3(256), 0, s, u, nrhs, st, nst, G, ld,
                     col0);
  return hipGetLastError();
}

hipError_t launch_lsq_lcurve(const double* G, const double* d, const double* L, const double* alphas, int32_t nobs,
                             int32_t nreg, int32_t nb, int32_t nalpha, double* work, double* a, double* rho,
                             double* eta, double* curv, int32_t* corner, hipStream_t s) {
  hipLaunchKernelGGL(k_lsq_qr, dim3(unsigned(nalpha)), dim3(kQrThreads), 0, s, G, d, L, alphas, nobs, nreg, nb, work,
                     a, rho, eta);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || nalpha < 3) return e;
  hipLaunchKernelGGL(k_lcurve_corner, dim3(1), dim3(256), 0, s, alphas, rho, eta, nalpha, curv, corner);
  return hipGetLastError();
}

}  // namespace ebe
