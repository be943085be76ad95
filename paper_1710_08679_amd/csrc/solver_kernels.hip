// Fused vector kernels of Algorithm 1 and their device-side scalar steps.
//
// Every CG loop in Algorithm 1 carries n cases with per-case scalars and
// stops when the worst case meets its test (Section 3.1).  Here those scalars
// never leave the GPU: a kernel that needs an inner product leaves per-case
// partial sums per workgroup, and a one-workgroup kernel after it adds them
// in a fixed order and runs the scalar step (alpha, beta, rho, the stopping
// test) for all cases.  Loop control is a device flag that
// every later kernel of the loop reads first, so the host can enqueue
// iterations ahead and only reads the flag now and then.
//
// Work unit = (node, case): a work-item reads the three components of one
// case of one node (stride n in the [node][component][case] layout), which
// the 3x3 block Jacobi needs; a workgroup holds a multiple of n work-items so
// each work-item keeps one case for the whole grid-stride loop.
#include <hip/hip_runtime.h>

#include "ebe_internal.h"
#include "solver_state.h"

namespace ebe {
namespace {

constexpr int kMaxBlocks = 1024;

__host__ __device__ constexpr int block_for(int nr) { return (256 / nr) * nr; }

template <typename T>
__device__ __forceinline__ void bj_apply(const T* __restrict__ m, T x0, T x1, T x2, T& y0, T& y1, T& y2) {
  y0 = m[0] * x0 + m[5] * x1 + m[4] * x2;
  y1 = m[5] * x0 + m[1] * x1 + m[3] * x2;
  y2 = m[4] * x0 + m[3] * x1 + m[2] * x2;
}

__device__ __forceinline__ bool finite_d(double v) { return isfinite(v); }

// ---------------------------------------------------------------------------
// generic node-case kernel with NDOT per-case inner products and an epilogue
// ---------------------------------------------------------------------------
// Each workgroup leaves its per-case sums in partials[output][workgroup]; a
// one-workgroup kernel launched right after adds them in a fixed order and
// runs the scalar step.  (A last-arriving-workgroup reduction inside the
// first kernel needs a device-scope fence in every workgroup, which on this
// multi-XCD part writes back the XCD's L2 each time: measured to cost about
// as much as the vector work itself on the linear level.  The kernel
// boundary makes the partials visible with one write-back.)
template <typename Acc, int NDOT, class Body>
__global__ __launch_bounds__(256) void k_nodecase(Body body, int64_t n_nodes, int nr, Acc* __restrict__ partials,
                                                  const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  // 256 work-items per workgroup; the first bd = (256 / nr) nr of them walk
  // the (node, case) units with a stride that is a multiple of nr, so each
  // keeps one case; the others only join the reductions.
  const int bd = block_for(nr);
  const int col = threadIdx.x % nr;
  Acc acc[NDOT > 0 ? NDOT : 1];
#pragma unroll
  for (int d = 0; d < (NDOT > 0 ? NDOT : 1); ++d) acc[d] = Acc(0);
  const int64_t units = n_nodes * nr;
  if (int(threadIdx.x) < bd) {
    // four units per trip, so each work-item has four units' loads in flight
    const int64_t stride = int64_t(gridDim.x) * bd;
    int64_t u = int64_t(blockIdx.x) * bd + threadIdx.x;
    for (; u + 3 * stride < units; u += 4 * stride) {
#pragma unroll
      for (int k = 0; k < 4; ++k) body((u + k * stride) / nr, col, acc);
    }
    for (; u < units; u += stride) body(u / nr, col, acc);
  }
  if constexpr (NDOT > 0) {
    __shared__ Acc sh[256 * NDOT];
#pragma unroll
    for (int d = 0; d < NDOT; ++d) sh[d * 256 + threadIdx.x] = acc[d];
    __syncthreads();
    const int nsum = NDOT * nr;
    if (threadIdx.x < nsum) {
      const int d = threadIdx.x / nr, c = threadIdx.x % nr;
      Acc s = Acc(0);
      for (int k = c; k < bd; k += nr) s += sh[d * 256 + k];
      partials[size_t(threadIdx.x) * kMaxBlocks + blockIdx.x] = s;
    }
  }
}

// Sum the partials of `blocks` workgroups with 256 work-items: output o gets
// partials b = t, t + 256, t + 512, t + 768 from work-item t (eight outputs'
// loads in flight at once), then a fixed-order wavefront tree and a sum over
// the 4 wavefronts (deterministic), and run the epilogue on the totals.
template <typename Acc, int NDOT, class Epi>
__global__ __launch_bounds__(256) void k_nodecase_epi(Epi epi, int nr, int blocks, const Acc* __restrict__ partials,
                                                      const int* __restrict__ gate) {
  static_assert(kMaxBlocks == 4 * 256, "four partials per work-item");
  if (gate && *gate == 0) return;
  __shared__ double tot[3 * EBE_MAX_RHS];
  __shared__ double wsum[4][3 * EBE_MAX_RHS];
  const int nsum = NDOT * nr;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // Every load reads a written partial (indices clamped to the last output
  // and workgroup), so all of them can be in flight together; the clamped
  // duplicates are then weighted by zero.  (A duplicate can only be
  // non-finite if an entry of the sum itself is, so the sum is unchanged.)
  for (int o0 = 0; o0 < nsum; o0 += 8) {
    double v[8][4];
#pragma unroll
    for (int j = 0; j < 8; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int b = int(threadIdx.x) + 256 * q;
        const int o = o0 + j;
        const double w = double(partials[size_t(o < nsum ? o : nsum - 1) * kMaxBlocks + (b < blocks ? b : blocks - 1)]);
        v[j][q] = w * ((o < nsum && b < blocks) ? 1.0 : 0.0);
      }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      double s = (v[j][0] + v[j][1]) + (v[j][2] + v[j][3]);
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
      if (lane == 0 && o0 + j < nsum) wsum[wave][o0 + j] = s;
    }
  }
  __syncthreads();
  if (int(threadIdx.x) < nsum)
    tot[threadIdx.x] = (wsum[0][threadIdx.x] + wsum[1][threadIdx.x]) + (wsum[2][threadIdx.x] + wsum[3][threadIdx.x]);
  __syncthreads();
  // per-case scalar steps on wavefront 0, the loop test's maximum and the
  // flags combined across it, then the shared step
  if (threadIdx.x < 64) {
    const int j = threadIdx.x;
    double worst = 0.0;
    int flags = 0;
    if (j < nr) worst = epi.step(tot, nr, j, flags);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      worst = fmax(worst, __shfl_xor(worst, off, 64));
      flags |= __shfl_xor(flags, off, 64);
    }
    if (j == 0) epi.finish(worst, flags);
  }
}

template <typename Acc, int NDOT, class Body, class Epi>
hipError_t run_nodecase(Body body, Epi epi, int64_t n_nodes, int nr, SolverState& st, const int* gate,
                        hipStream_t s) {
  const int bd = block_for(nr);
  int64_t g = (n_nodes * nr + bd - 1) / bd;
  if (g > kMaxBlocks) g = kMaxBlocks;
  if (g < 1) g = 1;
  Acc* partials = reinterpret_cast<Acc*>(st.partials);
  hipLaunchKernelGGL((k_nodecase<Acc, NDOT, Body>), dim3(unsigned(g)), dim3(256), 0, s, body, n_nodes, nr, partials,
                     gate);
  if constexpr (NDOT > 0) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_nodecase_epi<Acc, NDOT, Epi>), dim3(1), dim3(256), 0, s, epi, nr, int(g), partials, gate);
  }
  return hipGetLastError();
}

struct NoEpi {
  __device__ double step(const double*, int, int, int&) const { return 0.0; }
  __device__ void finish(double, int) const {}
};

// ---------------------------------------------------------------------------
// bodies
// ---------------------------------------------------------------------------
#define NC_IDX(node, c, col) ((node) * 3 * int64_t(nr) + (c) * nr + (col))

// u <- P u (fixed DOFs to zero); f is only read
struct BodyMaskU {
  double* u;
  const uint8_t* fix;
  int nr;
  __device__ void operator()(int64_t node, int col, double*) const {
    const unsigned fx = fix[node];
#pragma unroll
    for (int c = 0; c < 3; ++c)
      if ((fx >> c) & 1) u[NC_IDX(node, c, col)] = 0.0;
  }
};

// r = P f - q ; sums: ||Pf||^2, ||r||^2
struct BodyOuterInit {
  const double* f;
  const double* q;
  double* r;
  const uint8_t* fix;
  int nr;
  __device__ void operator()(int64_t node, int col, double* acc) const {
    const unsigned fx = fix[node];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int64_t i = NC_IDX(node, c, col);
      const double fv = ((fx >> c) & 1) ? 0.0 : f[i];
      const double rv = ((fx >> c) & 1) ? 0.0 : fv - q[i];
      r[i] = rv;
      acc[0] += fv * fv;
      acc[1] += rv * rv;
    }
  }
};

// The outer preconditioned residual z is never stored: it is M^-1 r (PCGE)
// or the preconditioner's output u_bar (MG2), recomputed or read where used.
template <int MODE, typename TU>
struct OuterZ {
  const double* minv;  // MODE 0: z = M^-1 r
  const TU* ub;        // MODE 1: z = (double) u_bar
  __device__ __forceinline__ void operator()(int64_t node, int64_t i0, int nr, double r0, double r1, double r2,
                                             double& z0, double& z1, double& z2) const {
    if (MODE == 0) {
      bj_apply(minv + 6 * node, r0, r1, r2, z0, z1, z2);
    } else {
      z0 = double(ub[i0]);
      z1 = double(ub[i0 + nr]);
      z2 = double(ub[i0 + 2 * nr]);
    }
  }
};

// sums: (z, q) with q the previous K p, and (z, r)
template <int MODE, typename TU>
struct BodyOuterZ {
  OuterZ<MODE, TU> zf;
  const double* r;
  const double* q;
  int nr;
  __device__ void operator()(int64_t node, int col, double* acc) const {
    const int64_t i0 = NC_IDX(node, 0, col);
    const double r0 = r[i0], r1 = r[i0 + nr], r2 = r[i0 + 2 * nr];
    double z0, z1, z2;
    zf(node, i0, nr, r0, r1, r2, z0, z1, z2);
    acc[0] += z0 * q[i0] + z1 * q[i0 + nr] + z2 * q[i0 + 2 * nr];
    acc[1] += z0 * r0 + z1 * r1 + z2 * r2;
  }
};

// p = z + beta p (z recomputed as above)
template <int MODE, typename TU>
struct BodyOuterP {
  OuterZ<MODE, TU> zf;
  const double* r;
  double* p;
  const double* beta;
  int nr;
  __device__ void operator()(int64_t node, int col, double*) const {
    const int64_t i0 = NC_IDX(node, 0, col);
    double z[3];
    zf(node, i0, nr, MODE == 0 ? r[i0] : 0.0, MODE == 0 ? r[i0 + nr] : 0.0, MODE == 0 ? r[i0 + 2 * nr] : 0.0,
       z[0], z[1], z[2]);
    const double b = beta[col];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int64_t i = i0 + c * nr;
      // beta = 0 starts a new direction: do not read p (it may hold stale bits)
      p[i] = (b == 0.0) ? z[c] : z[c] + b * p[i];
    }
  }
};

// CG step length alpha = rho / (p, K p).  The outer loop takes no step for a
// non-positive curvature (flagged as a breakdown in its scalar step); an
// inner column whose denominator vanished is frozen.
__device__ __forceinline__ double outer_alpha(double rho, double gamma) {
  const double a = gamma > 0.0 ? rho / gamma : 0.0;
  return isfinite(a) ? a : 0.0;
}
__device__ __forceinline__ double inner_alpha(double rho, double gamma) {
  const double a = gamma != 0.0 ? rho / gamma : 0.0;
  return isfinite(a) ? a : 0.0;
}

// r -= alpha q ; u += alpha p ; sums: ||r||^2   (alpha = rho / gamma per case;
// gamma = (p, K p) was accumulated by the product that formed q)
// WITH_Z (PCGE): also z = M^-1 r of the new residual, and the next step's
// sums (z, q) and (z, r), while r and q are at hand (sums: ||r||^2, (z, q),
// (z, r)); the separate z pass of the next iteration is then not needed.
template <bool WITH_Z>
struct BodyOuterUpdate {
  double* r;
  double* u;
  const double* q;
  const double* p;
  const double* minv;  // WITH_Z
  const SolverScalars* sc;
  int nr;
  __device__ void operator()(int64_t node, int col, double* acc) const {
    const double a = outer_alpha(sc->rho[col], sc->gamma[col]);
    double rv[3], qv[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int64_t i = NC_IDX(node, c, col);
      qv[c] = q[i];
      rv[c] = r[i] - a * qv[c];
      r[i] = rv[c];
      u[i] += a * p[i];
      acc[0] += rv[c] * rv[c];
    }
    if constexpr (WITH_Z) {
      double z0, z1, z2;
      bj_apply(minv + 6 * node, rv[0], rv[1], rv[2], z0, z1, z2);
      acc[1] += z0 * qv[0] + z1 * qv[1] + z2 * qv[2];
      acc[2] += z0 * rv[0] + z1 * rv[1] + z2 * rv[2];
    }
  }
};

// rb = (T) r ; ub = M0^-1 rb
template <typename T>
struct BodyCastBJ {
  const double* r;
  const T* minv;
  T* rb;
  T* ub;
  int nr;
  __device__ void operator()(int64_t node, int col, double*) const {
    const int64_t i0 = NC_IDX(node, 0, col);
    const T r0 = T(r[i0]), r1 = T(r[i0 + nr]), r2 = T(r[i0 + 2 * nr]);
    rb[i0] = r0;
    rb[i0 + nr] = r1;
    rb[i0 + 2 * nr] = r2;
    T y0, y1, y2;
    bj_apply(minv + 6 * node, r0, r1, r2, y0, y1, y2);
    ub[i0] = y0;
    ub[i0 + nr] = y1;
    ub[i0 + 2 * nr] = y2;
  }
};

// inner start: e = r - q ; sums ||e||^2, (M^-1 e, e), ||r||^2
template <typename T>
struct BodyInnerInit {
  const T* r;
  const T* q;
  T* e;
  const T* minv;
  int nr;
  __device__ void operator()(int64_t node, int col, T* acc) const {
    const int64_t i0 = NC_IDX(node, 0, col);
    const T r0 = r[i0], r1 = r[i0 + nr], r2 = r[i0 + 2 * nr];
    const T e0 = r0 - q[i0], e1 = r1 - q[i0 + nr], e2 = r2 - q[i0 + 2 * nr];
    e[i0] = e0;
    e[i0 + nr] = e1;
    e[i0 + 2 * nr] = e2;
    T z0, z1, z2;
    bj_apply(minv + 6 * node, e0, e1, e2, z0, z1, z2);
    acc[0] += e0 * e0 + e1 * e1 + e2 * e2;
    acc[1] += z0 * e0 + z1 * e1 + z2 * e2;
    acc[2] += r0 * r0 + r1 * r1 + r2 * r2;
  }
};

// p = M^-1 e + beta p ; q = 0
template <typename T>
struct BodyInnerP {
  const T* e;
  T* p;
  T* q;
  const T* minv;
  const double* beta;
  int nr;
  __device__ void operator()(int64_t node, int col, T*) const {
    const int64_t i0 = NC_IDX(node, 0, col);
    T z0, z1, z2;
    bj_apply(minv + 6 * node, e[i0], e[i0 + nr], e[i0 + 2 * nr], z0, z1, z2);
    const T b = T(beta[col]);
    if (b == T(0)) {  // first step of the loop: p may hold stale bits
      p[i0] = z0;
      p[i0 + nr] = z1;
      p[i0 + 2 * nr] = z2;
    } else {
      p[i0] = z0 + b * p[i0];
      p[i0 + nr] = z1 + b * p[i0 + nr];
      p[i0 + 2 * nr] = z2 + b * p[i0 + 2 * nr];
    }
  }
};

// e -= alpha q ; u += alpha p ; sums ||e||^2, (M^-1 e, e)
template <typename T>
struct BodyInnerUpdate {
  T* e;
  T* u;
  const T* q;
  const T* p;
  const T* minv;
  const InnerScalars* in;
  int nr;
  __device__ void operator()(int64_t node, int col, T* acc) const {
    const int64_t i0 = NC_IDX(node, 0, col);
    const T a = T(inner_alpha(in->rho_a[col], in->gamma[col]));
    T ev[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int64_t i = i0 + c * nr;
      ev[c] = e[i] - a * q[i];
      e[i] = ev[c];
      u[i] += a * p[i];
    }
    T z0, z1, z2;
    bj_apply(minv + 6 * node, ev[0], ev[1], ev[2], z0, z1, z2);
    acc[0] += ev[0] * ev[0] + ev[1] * ev[1] + ev[2] * ev[2];
    acc[1] += z0 * ev[0] + z1 * ev[1] + z2 * ev[2];
  }
};

// sums (a, b) per case in FP64 (the (p, K p) of a deterministic solve)
template <typename T>
struct BodyDot {
  const T* a;
  const T* b;
  int nr;
  __device__ void operator()(int64_t node, int col, double* acc) const {
    const int64_t i0 = NC_IDX(node, 0, col);
    acc[0] += double(a[i0]) * double(b[i0]) + double(a[i0 + nr]) * double(b[i0 + nr]) +
              double(a[i0 + 2 * nr]) * double(b[i0 + 2 * nr]);
  }
};

#undef NC_IDX

// ---------------------------------------------------------------------------
// epilogues (run by one thread of the last workgroup); see solver_state.h
// ---------------------------------------------------------------------------
// Epilogues run in two parts: step(tot, nr, j, flags) on work-item j for each
// case j < nr (returns the case's value for the loop test's maximum and may
// raise flag bits), then finish(worst, flags) once with the maximum and the
// union of the flags.  kBreakdown / kNonfinite: (p, K p) <= 0 for a live
// case, or a non-finite scalar (the latter takes precedence).
constexpr int kBreakdown = 1, kNonfinite = 2;

__device__ __forceinline__ int error_of(int flags) {
  return (flags & kNonfinite) ? EBE_ERR_NONFINITE : ((flags & kBreakdown) ? EBE_ERR_BREAKDOWN : 0);
}

struct EpiOuterInit {
  SolverScalars* sc;
  double tol;
  __device__ double step(const double* tot, int nr, int j, int& flags) const {
    const double ff = tot[j], rr = tot[nr + j];
    sc->nf2[j] = ff;
    sc->rr[j] = rr;
    const double rel = ff > 0.0 ? sqrt(rr / ff) : 0.0;
    sc->rel[j] = rel;
    if (!finite_d(rel) || !finite_d(ff) || !finite_d(rr)) flags |= kNonfinite;
    sc->alpha[j] = 0.0;
    sc->beta[j] = 0.0;
    sc->rho[j] = 0.0;
    return rel;
  }
  __device__ void finish(double worst, int flags) const {
    sc->max_rel = worst;
    sc->outer_iter = 0;
    if (flags) sc->err = error_of(flags);
    sc->outer_active = (!flags && worst > tol) ? 1 : 0;
  }
};

struct EpiOuterBeta {
  SolverScalars* sc;
  __device__ double step(const double* tot, int nr, int j, int&) const {
    const double zq = tot[j], zr = tot[nr + j];
    // flexible CG: beta_i = -alpha_{i-1} (z_i, q_{i-1}) / rho_{i-1}
    double b = 0.0;
    if (sc->outer_iter != 0 && sc->rho[j] != 0.0) b = -sc->alpha[j] * zq / sc->rho[j];
    if (!finite_d(b)) b = 0.0;
    sc->beta[j] = b;
    sc->rho[j] = zr;
    return 0.0;
  }
  __device__ void finish(double, int) const {}
};

// scalar step after r -= alpha q, u += alpha p: record alpha (used by the next
// beta), check the curvature (p, K p), clear its accumulator, test convergence
struct EpiOuterConv {
  SolverScalars* sc;
  double tol;
  int max_outer;
  __device__ double step(const double* tot, int nr, int j, int& flags) const {
    const double g = sc->gamma[j];
    if (g < 0.0 || (g == 0.0 && sc->rr[j] > 0.0 && sc->rho[j] != 0.0)) flags |= kBreakdown;
    if (!finite_d(g)) flags |= kNonfinite;
    sc->alpha[j] = outer_alpha(sc->rho[j], g);
    sc->gamma[j] = 0.0;
    const double rr = tot[j];
    sc->rr[j] = rr;
    const double rel = sc->nf2[j] > 0.0 ? sqrt(rr / sc->nf2[j]) : 0.0;
    sc->rel[j] = rel;
    if (!finite_d(rel)) flags |= kNonfinite;
    return rel;
  }
  __device__ void finish(double worst, int flags) const {
    sc->max_rel = worst;
    sc->outer_iter += 1;
    if (flags) sc->err = error_of(flags);
    sc->outer_active = (!flags && !sc->err && worst > tol && sc->outer_iter < max_outer) ? 1 : 0;
  }
};

// EpiOuterConv followed by the next iteration's EpiOuterBeta (PCGE with the
// z sums formed in the update): beta_{i+1} = -alpha_i (z_{i+1}, q_i) / rho_i
// with the alpha just recorded, rho_{i+1} = (z_{i+1}, r_{i+1}).
struct EpiOuterConvBeta {
  EpiOuterConv conv;
  __device__ double step(const double* tot, int nr, int j, int& flags) const {
    const double rel = conv.step(tot, nr, j, flags);
    SolverScalars* sc = conv.sc;
    const double zq = tot[nr + j], zr = tot[2 * nr + j];
    double b = sc->rho[j] != 0.0 ? -sc->alpha[j] * zq / sc->rho[j] : 0.0;
    if (!finite_d(b)) b = 0.0;
    sc->beta[j] = b;
    sc->rho[j] = zr;
    return rel;
  }
  __device__ void finish(double worst, int flags) const { conv.finish(worst, flags); }
};

// gamma[j] = the case's sum (fixed-order partials; no atomics)
struct EpiSetGamma {
  double* gamma;
  __device__ double step(const double* tot, int, int j, int&) const {
    gamma[j] = tot[j];
    return 0.0;
  }
  __device__ void finish(double, int) const {}
};

template <typename T>
struct EpiInnerStart {
  InnerScalars* in;
  double eps;
  int nmax;
  __device__ double step(const double* tot, int nr, int j, int&) const {
    const double ee = tot[j], ze = tot[nr + j], rr = tot[2 * nr + j];
    in->nr2[j] = rr;
    const double ratio = rr > 0.0 ? ee / rr : 0.0;
    in->rho_a[j] = ze;
    in->beta[j] = 0.0;
    in->alpha[j] = 0.0;
    in->gamma[j] = 0.0;
    return isfinite(ratio) ? ratio : 0.0;
  }
  __device__ void finish(double worst, int) const {
    in->i = 1;
    in->active = (worst > eps && 1 < nmax) ? 1 : 0;
  }
};

// scalar step after e -= alpha q, u += alpha p: beta = rho_a(new) / rho_a(old)
// (a column with rho_a(old) = 0 restarts), clear the (p, K p) accumulator
template <typename T>
struct EpiInnerStep {
  InnerScalars* in;
  double eps;
  int nmax;
  __device__ double step(const double* tot, int nr, int j, int&) const {
    const double ee = tot[j], ze = tot[nr + j];
    const double ratio = in->nr2[j] > 0.0 ? ee / in->nr2[j] : 0.0;
    const double rho_old = in->rho_a[j];
    in->alpha[j] = inner_alpha(rho_old, in->gamma[j]);
    in->gamma[j] = 0.0;
    double b = (rho_old != 0.0) ? ze / rho_old : 0.0;
    if (!isfinite(b)) b = 0.0;
    in->beta[j] = b;
    in->rho_a[j] = ze;
    return isfinite(ratio) ? ratio : 0.0;
  }
  __device__ void finish(double worst, int) const {
    const int i = in->i + 1;
    in->i = i;
    in->steps += 1;
    in->active = (worst > eps && i < nmax) ? 1 : 0;
  }
};

}  // namespace

// ---------------------------------------------------------------------------
// launchers used by solver.cpp
// ---------------------------------------------------------------------------
hipError_t sk_mask_u(const ebe_mesh* m, double* u, int nr, SolverState& st, hipStream_t s) {
  return run_nodecase<double, 0>(BodyMaskU{u, m->fix.as<uint8_t>(), nr}, NoEpi{}, m->n_nodes, nr, st, nullptr, s);
}

hipError_t sk_outer_init(const ebe_mesh* m, const double* f, const double* q, double* r, int nr, double tol,
                         SolverState& st, hipStream_t s) {
  return run_nodecase<double, 2>(BodyOuterInit{f, q, r, m->fix.as<uint8_t>(), nr}, EpiOuterInit{st.sc, tol},
                                 m->n_nodes, nr, st, nullptr, s);
}

hipError_t sk_outer_z_bj(const ebe_mesh* m, const double* r, const double* q, int nr, SolverState& st,
                         hipStream_t s) {
  BodyOuterZ<0, double> b{{m->minv64[0].as<double>(), nullptr}, r, q, nr};
  return run_nodecase<double, 2>(b, EpiOuterBeta{st.sc}, m->n_nodes, nr, st, &st.sc->outer_active, s);
}

template <typename T>
hipError_t sk_outer_z_cast(const ebe_mesh* m, const T* ub, const double* r, const double* q, int nr,
                           SolverState& st, hipStream_t s) {
  BodyOuterZ<1, T> b{{nullptr, ub}, r, q, nr};
  return run_nodecase<double, 2>(b, EpiOuterBeta{st.sc}, m->n_nodes, nr, st, &st.sc->outer_active, s);
}
template hipError_t sk_outer_z_cast<float>(const ebe_mesh*, const float*, const double*, const double*, int,
                                           SolverState&, hipStream_t);
template hipError_t sk_outer_z_cast<double>(const ebe_mesh*, const double*, const double*, const double*, int,
                                            SolverState&, hipStream_t);

hipError_t sk_outer_p_bj(const ebe_mesh* m, const double* r, double* p, int nr, SolverState& st, hipStream_t s) {
  BodyOuterP<0, double> b{{m->minv64[0].as<double>(), nullptr}, r, p, st.sc->beta, nr};
  return run_nodecase<double, 0>(b, NoEpi{}, m->n_nodes, nr, st, &st.sc->outer_active, s);
}

template <typename T>
hipError_t sk_outer_p_cast(const ebe_mesh* m, const T* ub, double* p, int nr, SolverState& st, hipStream_t s) {
  BodyOuterP<1, T> b{{nullptr, ub}, nullptr, p, st.sc->beta, nr};
  return run_nodecase<double, 0>(b, NoEpi{}, m->n_nodes, nr, st, &st.sc->outer_active, s);
}
template hipError_t sk_outer_p_cast<float>(const ebe_mesh*, const float*, double*, int, SolverState&, hipStream_t);
template hipError_t sk_outer_p_cast<double>(const ebe_mesh*, const double*, double*, int, SolverState&,
                                            hipStream_t);

hipError_t sk_outer_update(const ebe_mesh* m, double* r, double* u, const double* q, const double* p, int nr,
                           double tol, int max_outer, SolverState& st, hipStream_t s) {
  return run_nodecase<double, 1>(BodyOuterUpdate<false>{r, u, q, p, nullptr, st.sc, nr},
                                 EpiOuterConv{st.sc, tol, max_outer}, m->n_nodes, nr, st, &st.sc->outer_active, s);
}

hipError_t sk_outer_update_z_bj(const ebe_mesh* m, double* r, double* u, const double* q, const double* p, int nr,
                                double tol, int max_outer, SolverState& st, hipStream_t s) {
  return run_nodecase<double, 3>(BodyOuterUpdate<true>{r, u, q, p, m->minv64[0].as<double>(), st.sc, nr},
                                 EpiOuterConvBeta{EpiOuterConv{st.sc, tol, max_outer}}, m->n_nodes, nr, st,
                                 &st.sc->outer_active, s);
}

template <typename T>
hipError_t sk_cast_bj(const ebe_mesh* m, const double* r, T* rb, T* ub, int nr, SolverState& st, hipStream_t s) {
  const T* minv = sizeof(T) == 8 ? reinterpret_cast<const T*>(m->minv64[0].as<void>())
                                 : reinterpret_cast<const T*>(m->minv32[0].as<void>());
  return run_nodecase<double, 0>(BodyCastBJ<T>{r, minv, rb, ub, nr}, NoEpi{}, m->n_nodes, nr, st,
                                 &st.sc->outer_active, s);
}
template hipError_t sk_cast_bj<float>(const ebe_mesh*, const double*, float*, float*, int, SolverState&, hipStream_t);
template hipError_t sk_cast_bj<double>(const ebe_mesh*, const double*, double*, double*, int, SolverState&,
                                       hipStream_t);

template <typename T>
static const T* minv_of(const ebe_mesh* m, int level) {
  return sizeof(T) == 8 ? reinterpret_cast<const T*>(m->minv64[level].as<void>())
                        : reinterpret_cast<const T*>(m->minv32[level].as<void>());
}

template <typename T>
hipError_t sk_inner_init(const ebe_mesh* m, int level, const T* r, const T* q, T* e, int nr, double eps, int nmax,
                         SolverState& st, hipStream_t s) {
  const int64_t n = level_rows(m, level);
  return run_nodecase<T, 3>(BodyInnerInit<T>{r, q, e, minv_of<T>(m, level), nr},
                            EpiInnerStart<T>{&st.sc->inner[level], eps, nmax}, n, nr, st, &st.sc->outer_active, s);
}

template <typename T>
hipError_t sk_inner_p(const ebe_mesh* m, int level, const T* e, T* p, T* q, int nr, SolverState& st,
                      hipStream_t s) {
  const int64_t n = level_rows(m, level);
  return run_nodecase<T, 0>(BodyInnerP<T>{e, p, q, minv_of<T>(m, level), st.sc->inner[level].beta, nr}, NoEpi{},
                            n, nr, st, &st.sc->inner[level].active, s);
}

template <typename T>
hipError_t sk_inner_update(const ebe_mesh* m, int level, T* e, T* u, const T* q, const T* p, int nr, double eps,
                           int nmax, SolverState& st, hipStream_t s) {
  const int64_t n = level_rows(m, level);
  return run_nodecase<T, 2>(BodyInnerUpdate<T>{e, u, q, p, minv_of<T>(m, level), &st.sc->inner[level], nr},
                            EpiInnerStep<T>{&st.sc->inner[level], eps, nmax}, n, nr, st,
                            &st.sc->inner[level].active, s);
}

template <typename T>
hipError_t sk_dot(const ebe_mesh* m, int level, const T* a, const T* b, int nr, double* gamma, const int* gate,
                  SolverState& st, hipStream_t s) {
  return run_nodecase<double, 1>(BodyDot<T>{a, b, nr}, EpiSetGamma{gamma}, level_rows(m, level), nr, st, gate, s);
}
template hipError_t sk_dot<float>(const ebe_mesh*, int, const float*, const float*, int, double*, const int*,
                                  SolverState&, hipStream_t);
template hipError_t sk_dot<double>(const ebe_mesh*, int, const double*, const double*, int, double*, const int*,
                                   SolverState&, hipStream_t);

#define EBE_INST(T)                                                                                              \
  template hipError_t sk_inner_init<T>(const ebe_mesh*, int, const T*, const T*, T*, int, double, int,            \
                                       SolverState&, hipStream_t);                                               \
  template hipError_t sk_inner_p<T>(const ebe_mesh*, int, const T*, T*, T*, int, SolverState&, hipStream_t);      \
  template hipError_t sk_inner_update<T>(const ebe_mesh*, int, T*, T*, const T*, const T*, int, double, int,       \
                                         SolverState&, hipStream_t);
EBE_INST(float)
EBE_INST(double)
#undef EBE_INST

}  // namespace ebe
