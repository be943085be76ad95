// Set-up kernels: nodal 3x3 diagonal blocks of K and K1 and their inverses
// ("diag[ ]" of Algorithm 1), Lame parameters, material checks, clearing.
#include <hip/hip_runtime.h>

#include "ebe_internal.h"
#include "p2_element.h"

namespace ebe {
namespace {

__device__ __forceinline__ void atomic_add(double* p, double v) { unsafeAtomicAdd(p, v); }

constexpr int kBlock = 256;

inline unsigned grid_for(int64_t work, int block = kBlock) {
  int64_t g = (work + block - 1) / block;
  return unsigned(g < 1 ? 1 : g);
}

// ---------------------------------------------------------------------------
// nodal 3x3 diagonal blocks (symmetric, 6 values), FP64
//   K_aa = (lambda + mu) M_a + mu tr(M_a) I,  M_a = int grad N_a grad N_a^T dV
//   quadratic corner i:  M = 3V/5 G_i G_i^T
//   quadratic edge (i,j): M = 4V/5 (2 G_i G_i^T + G_i G_j^T + G_j G_i^T + 2 G_j G_j^T)
//   linear corner i:     M = V G_i G_i^T
// ---------------------------------------------------------------------------
__device__ __forceinline__ void add_block(double* blk, const double M[6], double lam, double mu) {
  const double tr = M[0] + M[1] + M[2];
  const double lm = lam + mu;
  atomic_add(blk + 0, lm * M[0] + mu * tr);
  atomic_add(blk + 1, lm * M[1] + mu * tr);
  atomic_add(blk + 2, lm * M[2] + mu * tr);
  atomic_add(blk + 3, lm * M[3]);
  atomic_add(blk + 4, lm * M[4]);
  atomic_add(blk + 5, lm * M[5]);
}

__device__ __forceinline__ void outer_sym(const double a[3], const double b[3], double s, double M[6]) {
  // M += s * (a b^T + b a^T) / 2 stored as (xx yy zz yz zx xy)
  M[0] += s * a[0] * b[0];
  M[1] += s * a[1] * b[1];
  M[2] += s * a[2] * b[2];
  M[3] += s * 0.5 * (a[1] * b[2] + a[2] * b[1]);
  M[4] += s * 0.5 * (a[2] * b[0] + a[0] * b[2]);
  M[5] += s * 0.5 * (a[0] * b[1] + a[1] * b[0]);
}

template <int LEVEL>
__global__ __launch_bounds__(kBlock) void k_diag_blocks(const int32_t* __restrict__ conn,
                                                        const double4* __restrict__ xv,
                                                        const double2* __restrict__ lame,
                                                        double* __restrict__ blk, int64_t nelem) {
  const int64_t e = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (e >= nelem) return;
  int32_t cw[10];
#pragma unroll
  for (int a = 0; a < 10; ++a) cw[a] = conn[e * 10 + a] & kIdxMask;
  double G[4][3];
  const double V = tet_geometry<double>(xv[cw[0]], xv[cw[1]], xv[cw[2]], xv[cw[3]], G);
  const double2 lm = lame[e];
  if (LEVEL == 1) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      double M[6] = {0, 0, 0, 0, 0, 0};
      outer_sym(G[i], G[i], V, M);
      add_block(blk + size_t(cw[i]) * 6, M, lm.x, lm.y);
    }
    return;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    double M[6] = {0, 0, 0, 0, 0, 0};
    outer_sym(G[i], G[i], 0.6 * V, M);
    add_block(blk + size_t(cw[i]) * 6, M, lm.x, lm.y);
  }
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    const int i = edge_end(q, 0), j = edge_end(q, 1);
    double M[6] = {0, 0, 0, 0, 0, 0};
    const double s = 0.8 * V;
    outer_sym(G[i], G[i], 2.0 * s, M);
    outer_sym(G[j], G[j], 2.0 * s, M);
    outer_sym(G[i], G[j], 2.0 * s, M);  // G_i G_j^T + G_j G_i^T
    add_block(blk + size_t(cw[4 + q]) * 6, M, lm.x, lm.y);
  }
}

// Quadratic-level blocks of curved elements: M_a = sum_q (det J_q / 24)
// g_aq g_aqᵀ with g_aq = grad N_a at quadrature point q (p2_element.h: the
// barycentric derivatives of N_a against the point's gradients grad L_k).
__global__ __launch_bounds__(kBlock) void k_diag_blocks_curved(const int32_t* __restrict__ conn,
                                                               const double4* __restrict__ xv,
                                                               const double2* __restrict__ lame,
                                                               double* __restrict__ blk, int64_t nelem) {
  const int64_t e = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (e >= nelem) return;
  int32_t cw[10];
  double d[10][3];
#pragma unroll
  for (int a = 0; a < 10; ++a) cw[a] = conn[e * 10 + a] & kIdxMask;
  const double4 x0 = xv[cw[0]];
#pragma unroll
  for (int a = 0; a < 10; ++a) {
    const double4 xa = xv[cw[a]];
    d[a][0] = xa.x - x0.x;
    d[a][1] = xa.y - x0.y;
    d[a][2] = xa.z - x0.z;
  }
  double M[10][6];
#pragma unroll
  for (int a = 0; a < 10; ++a)
#pragma unroll
    for (int c = 0; c < 6; ++c) M[a][c] = 0.0;
#pragma unroll 1
  for (int q = 0; q < 4; ++q) {
    double G[3][3], Gk[4][3];
    const double w = curved_point(d, q, G) * (1.0 / 24.0);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      Gk[1][c] = G[0][c];
      Gk[2][c] = G[1][c];
      Gk[3][c] = G[2][c];
      Gk[0][c] = -((G[0][c] + G[1][c]) + G[2][c]);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const double ck = 4.0 * quad_l(q, k) - 1.0;
      const double g[3] = {ck * Gk[k][0], ck * Gk[k][1], ck * Gk[k][2]};
      outer_sym(g, g, w, M[k]);
    }
#pragma unroll
    for (int ed = 0; ed < 6; ++ed) {
      const int k = edge_end(ed, 0), m = edge_end(ed, 1);
      const double lm = 4.0 * quad_l(q, m), lk = 4.0 * quad_l(q, k);
      double g[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) g[c] = lm * Gk[k][c] + lk * Gk[m][c];
      outer_sym(g, g, w, M[4 + ed]);
    }
  }
  const double2 lm = lame[e];
#pragma unroll
  for (int a = 0; a < 10; ++a) add_block(blk + size_t(cw[a]) * 6, M[a], lm.x, lm.y);
}

// fixed DOFs -> identity rows/columns, then invert (symmetric 3x3, FP64)
__global__ __launch_bounds__(kBlock) void k_invert_blocks(const double* __restrict__ blk,
                                                          const uint8_t* __restrict__ fix,
                                                          double* __restrict__ inv64,
                                                          float* __restrict__ inv32, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= n) return;
  double a[3][3];
  const double* b = blk + 6 * i;
  a[0][0] = b[0]; a[1][1] = b[1]; a[2][2] = b[2];
  a[1][2] = a[2][1] = b[3];
  a[2][0] = a[0][2] = b[4];
  a[0][1] = a[1][0] = b[5];
  const unsigned fx = fix[i];
#pragma unroll
  for (int c = 0; c < 3; ++c)
    if ((fx >> c) & 1) {
#pragma unroll
      for (int d = 0; d < 3; ++d) a[c][d] = a[d][c] = 0.0;
      a[c][c] = 1.0;
    }
  const double c00 = a[1][1] * a[2][2] - a[1][2] * a[2][1];
  const double c01 = a[1][2] * a[2][0] - a[1][0] * a[2][2];
  const double c02 = a[1][0] * a[2][1] - a[1][1] * a[2][0];
  const double det = a[0][0] * c00 + a[0][1] * c01 + a[0][2] * c02;
  const double id = 1.0 / det;
  double o[6];
  o[0] = c00 * id;
  o[1] = (a[0][0] * a[2][2] - a[0][2] * a[2][0]) * id;
  o[2] = (a[0][0] * a[1][1] - a[0][1] * a[1][0]) * id;
  o[3] = (a[0][2] * a[1][0] - a[0][0] * a[1][2]) * id;  // yz
  o[4] = c02 * id;                                        // zx
  o[5] = c01 * id;                                        // xy
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    inv64[6 * i + c] = o[c];
    inv32[6 * i + c] = float(o[c]);
  }
}

__global__ __launch_bounds__(kBlock) void k_expand_blocks(const double* __restrict__ b6,
                                                          double* __restrict__ b9, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= n) return;
  const double* b = b6 + 6 * i;
  double* o = b9 + 9 * i;
  o[0] = b[0]; o[1] = b[5]; o[2] = b[4];
  o[3] = b[5]; o[4] = b[1]; o[5] = b[3];
  o[6] = b[4]; o[7] = b[3]; o[8] = b[2];
}

__global__ __launch_bounds__(kBlock) void k_lame(const double* __restrict__ E,
                                                 const double* __restrict__ nu,
                                                 double2* __restrict__ l64, float2* __restrict__ l32,
                                                 int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= n) return;
  const double e = E[i], v = nu[i];
  const double lam = e * v / ((1.0 + v) * (1.0 - 2.0 * v));
  const double mu = e / (2.0 * (1.0 + v));
  l64[i] = make_double2(lam, mu);
  l32[i] = make_float2(float(lam), float(mu));
}

// Geometry cache row of element i: barycentric gradients G (4 x 3), volume
// V, lambda, mu (then padding to 16 values), formed exactly as the patch
// kernels form them from the corner coordinates.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_geometry(const int32_t* __restrict__ conn, const double4* __restrict__ xv,
                                                     const double2* __restrict__ lame, T* __restrict__ out,
                                                     int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= n) return;
  T G[4][3];
  const T V = tet_geometry<T>(xv[conn[i * 10 + 0] & kIdxMask], xv[conn[i * 10 + 1] & kIdxMask],
                              xv[conn[i * 10 + 2] & kIdxMask], xv[conn[i * 10 + 3] & kIdxMask], G);
  T* o = out + i * 16;
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int d = 0; d < 3; ++d) o[3 * k + d] = G[k][d];
  const double2 lm = lame[i];
  o[12] = V;
  o[13] = T(lm.x);
  o[14] = T(lm.y);
  o[15] = T(0);
}

// Level-2 prolongator P2 = (I - omega D1^-1 K1p) T, one work-item per fine
// row v: slot w of the row (aggregate J) is [J = agg(v)] I_free(v)
// - omega D1^-1(v) sum_{b in row v of K1, agg(b) = J} K1p(v, b), with K1p's
// fixed rows and columns left out and D1^-1 the level-1 block-Jacobi inverse
// (identity at fixed DOFs).  The sums are accumulated in the output row.
constexpr double kOmega = 2.0 / 3.0;

__global__ __launch_bounds__(kBlock) void k_smooth_p2(const int32_t* __restrict__ k1soff,
                                                      const int32_t* __restrict__ k1col,
                                                      const double* __restrict__ k1val,
                                                      const uint8_t* __restrict__ fix,
                                                      const int32_t* __restrict__ agg,
                                                      const double* __restrict__ minv1,
                                                      const int32_t* __restrict__ pcol, int width,
                                                      double* __restrict__ p64, float* __restrict__ p32,
                                                      int64_t nv) {
  constexpr int S = kSliceRows;
  const int64_t v = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (v >= nv) return;
  const int64_t sl = v / S;
  const int r = int(v - sl * S);
  const int fa = fix[v];
  const int32_t* pc = pcol + size_t(v) * width;
  double* out = p64 + size_t(v) * width * 9;
  for (int i = 0; i < width * 9; ++i) out[i] = 0.0;
  for (int32_t j = k1soff[sl]; j < k1soff[sl + 1]; ++j) {
    const int32_t wd = k1col[size_t(j) * S + r];
    const int fb = (wd >> kIdxBits) & 7;
    const int32_t J = agg[wd & kIdxMask];
    int w = 0;
    while (w < width - 1 && pc[w] != J) ++w;
    if (pc[w] != J) continue;  // cannot happen: the row lists every neighbour's aggregate
    const double* blk = k1val + size_t(j) * 9 * S + r;
    for (int p = 0; p < 3; ++p)
      for (int q = 0; q < 3; ++q)
        if (!((fa >> p) & 1) && !((fb >> q) & 1)) out[w * 9 + 3 * p + q] += blk[(3 * p + q) * S];
  }
  const double* m = minv1 + 6 * v;
  const double D[3][3] = {{m[0], m[5], m[4]}, {m[5], m[1], m[3]}, {m[4], m[3], m[2]}};
  const int32_t av = agg[v];
  for (int w = 0; w < width; ++w) {
    double B[9];
    for (int i = 0; i < 9; ++i) B[i] = out[w * 9 + i];
    for (int p = 0; p < 3; ++p)
      for (int q = 0; q < 3; ++q) {
        double val = (pc[w] == av && p == q && !((fa >> p) & 1)) ? 1.0 : 0.0;
        val -= kOmega * (D[p][0] * B[q] + D[p][1] * B[3 + q] + D[p][2] * B[6 + q]);
        out[w * 9 + 3 * p + q] = val;
        p32[size_t(v) * width * 9 + w * 9 + 3 * p + q] = float(val);
      }
  }
}

// A2 = P2^T K1p P2 by coarse rows, without global atomics: one wavefront per
// row I of A2 walks the P2 entries (v, I) (the transposed prolongator) and
// v's K1 blocks (v, b), and adds P2(v, I)^T K1p(v, b) P2(b, J) for every
// slot J of P2's row b into the row's blocks held in LDS (columns found by
// bisection in the row's column list), then writes the row.  Level 2 is
// refused (MG2 remains) on a mesh whose longest A2 row does not fit the LDS.
constexpr int kGalerkinThreads = 64;
constexpr int kGalerkinMaxRow = kA2MaxRow;

__global__ __launch_bounds__(kGalerkinThreads) void k_galerkin_rows(
    const int32_t* __restrict__ k1soff, const int32_t* __restrict__ k1col, const double* __restrict__ k1val,
    const uint8_t* __restrict__ fix, const int32_t* __restrict__ pcol, int width, const double* __restrict__ p64,
    const int32_t* __restrict__ toff, const int32_t* __restrict__ tidx, const int32_t* __restrict__ a2soff,
    const int32_t* __restrict__ a2col, const int32_t* __restrict__ a2len, double* __restrict__ a2val,
    int64_t na) {
  constexpr int S = kSliceRows;
  extern __shared__ double lds[];  // [len][9] block sums, then [len] column ids
  const int64_t I = blockIdx.x;
  if (I >= na) return;
  const int tid = threadIdx.x;
  const int64_t sI = I / S;
  const int rI = int(I - sI * S);
  const int len = a2len[I];
  const int32_t k0 = a2soff[sI];
  double* acc = lds;
  int32_t* cols = reinterpret_cast<int32_t*>(lds + size_t(len) * 9);
  for (int i = tid; i < len; i += kGalerkinThreads) cols[i] = a2col[size_t(k0 + i) * S + rI] & kIdxMask;
  for (int i = tid; i < len * 9; i += kGalerkinThreads) acc[i] = 0.0;
  __syncthreads();
  for (int32_t t = toff[I] + tid; t < toff[I + 1]; t += kGalerkinThreads) {
    const int64_t e = tidx[t];
    const int64_t v = e / width;
    const double* PI = p64 + e * 9;
    const int fa = fix[v];
    const int64_t sl = v / S;
    const int r = int(v - sl * S);
    for (int32_t j = k1soff[sl]; j < k1soff[sl + 1]; ++j) {
      const int32_t wd = k1col[size_t(j) * S + r];
      const int fb = (wd >> kIdxBits) & 7;
      const int64_t b = wd & kIdxMask;
      const double* blk = k1val + size_t(j) * 9 * S + r;
      double T[3][3];
      bool any = false;
      for (int p = 0; p < 3; ++p)
        for (int q = 0; q < 3; ++q) {
          T[p][q] = (!((fa >> p) & 1) && !((fb >> q) & 1)) ? blk[(3 * p + q) * S] : 0.0;
          any |= T[p][q] != 0.0;
        }
      if (!any) continue;
      double L[3][3];  // P2(v, I)^T K1p(v, b)
      for (int p = 0; p < 3; ++p)
        for (int q = 0; q < 3; ++q) L[p][q] = PI[0 * 3 + p] * T[0][q] + PI[1 * 3 + p] * T[1][q] + PI[2 * 3 + p] * T[2][q];
      for (int wj = 0; wj < width; ++wj) {
        const int32_t J = pcol[b * width + wj];
        if (J < 0) break;
        int lo = 0, hi = len - 1;
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (cols[mid] < J) lo = mid + 1;
          else hi = mid;
        }
        if (cols[lo] != J) continue;  // cannot happen (structure)
        const double* PJ = p64 + (b * width + wj) * 9;
        for (int p = 0; p < 3; ++p)
          for (int q = 0; q < 3; ++q)
            atomicAdd(acc + lo * 9 + 3 * p + q, L[p][0] * PJ[0 * 3 + q] + L[p][1] * PJ[1 * 3 + q] + L[p][2] * PJ[2 * 3 + q]);
      }
    }
  }
  __syncthreads();
  for (int i = tid; i < len * 9; i += kGalerkinThreads)
    a2val[(size_t(k0 + i / 9) * 9 + i % 9) * S + rI] = acc[i];
}

// diagonal 3x3 blocks of an assembled operator as (xx yy zz yz zx xy)
__global__ __launch_bounds__(kBlock) void k_asm_diag(const int32_t* __restrict__ soff,
                                                     const int32_t* __restrict__ col,
                                                     const double* __restrict__ val, double* __restrict__ blk,
                                                     int64_t n) {
  constexpr int S = kSliceRows;
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= n) return;
  const int64_t sl = i / S;
  const int r = int(i - sl * S);
  double* b = blk + 6 * i;
  for (int k = 0; k < 6; ++k) b[k] = 0.0;
  for (int32_t j = soff[sl]; j < soff[sl + 1]; ++j)
    if ((col[size_t(j) * S + r] & kIdxMask) == i) {
      const double* v = val + size_t(j) * 9 * S + r;
      b[0] = v[0 * S];
      b[1] = v[4 * S];
      b[2] = v[8 * S];
      b[3] = v[5 * S];
      b[4] = v[2 * S];
      b[5] = v[1 * S];
      return;
    }
}

// K1 by rows, without atomics: one work-item per corner v writes its row's
// blocks, summing for each element around v (the corner's element list,
// each entry element * 4 + local corner a) the blocks (a, b) of the linear
// tetrahedron, V [lambda G_a G_b^T + mu (G_a . G_b) I + mu G_b G_a^T]
// (f_a = V sigma G_a with sigma from the constant strain; the operator
// p1_forces applies), each found in the row by a scan of its (short) slot
// list; padding slots stay zero.  The rows of a wavefront are the 64
// rows of one slice, so each value access of the wavefront is one
// contiguous run.
__global__ __launch_bounds__(kBlock) void k_assemble_p1_rows(const int32_t* __restrict__ conn,
                                                             const double4* __restrict__ xv,
                                                             const double2* __restrict__ lame,
                                                             const int32_t* __restrict__ voff,
                                                             const int32_t* __restrict__ vel,
                                                             const int32_t* __restrict__ soff,
                                                             const int32_t* __restrict__ col,
                                                             double* __restrict__ val, int64_t nv) {
  constexpr int S = kSliceRows;
  const int64_t v = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (v >= nv) return;
  const int64_t sl = v / S;
  const int r = int(v - sl * S);
  const int32_t j0 = soff[sl], j1 = soff[sl + 1];
  for (int32_t j = j0; j < j1; ++j)
    for (int i = 0; i < 9; ++i) val[(size_t(j) * 9 + i) * S + r] = 0.0;
  for (int32_t t = voff[v]; t < voff[v + 1]; ++t) {
    const int64_t el = vel[t] >> 2;
    const int a = vel[t] & 3;
    int w[4];
    for (int k = 0; k < 4; ++k) w[k] = conn[el * 10 + k] & kIdxMask;
    double G[4][3];
    const double V = tet_geometry<double>(xv[w[0]], xv[w[1]], xv[w[2]], xv[w[3]], G);
    const double2 lm = lame[el];
    const double cl = lm.x * V, cm = lm.y * V;
    for (int b = 0; b < 4; ++b) {
      int32_t j = j0;
      while (j < j1 && (col[size_t(j) * S + r] & kIdxMask) != w[b]) ++j;
      if (j == j1) continue;  // cannot happen for a consistent structure
      const double gg = G[a][0] * G[b][0] + G[a][1] * G[b][1] + G[a][2] * G[b][2];
      double* blk = val + size_t(j) * 9 * S + r;
      for (int p = 0; p < 3; ++p)
        for (int q = 0; q < 3; ++q)
          blk[(3 * p + q) * S] += cl * G[a][p] * G[b][q] + cm * G[a][q] * G[b][p] + (p == q ? cm * gg : 0.0);
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_to_f32(const double* __restrict__ a, float* __restrict__ b, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock)
    b[i] = float(a[i]);
}

// largest |a_i| (non-negative doubles order as their bit patterns)
__global__ __launch_bounds__(kBlock) void k_absmax(const double* __restrict__ a, int64_t n,
                                                   unsigned long long* __restrict__ out) {
  double mx = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock)
    mx = fmax(mx, fabs(a[i]));
  for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
  if ((threadIdx.x & 63) == 0) atomicMax(out, static_cast<unsigned long long>(__double_as_longlong(mx)));
}

__global__ __launch_bounds__(kBlock) void k_to_f16(const double* __restrict__ a, _Float16* __restrict__ b, int64_t n,
                                                   double inv_scale) {
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock)
    b[i] = _Float16(float(a[i] * inv_scale));
}

__global__ __launch_bounds__(kBlock) void k_check_material(const double* __restrict__ E,
                                                           const double* __restrict__ nu,
                                                           int* __restrict__ bad, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= n) return;
  const double e = E[i], v = nu[i];
  const bool ok = isfinite(e) && isfinite(v) && e > 0.0 && v > -1.0 && v < 0.5;
  if (!ok) atomicAdd(bad, 1);
}

__global__ __launch_bounds__(kBlock) void k_fill_zero(uint32_t* __restrict__ p, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock)
    p[i] = 0u;
}

}  // namespace

hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s) {
  const int64_t n = int64_t(bytes / 4);
  if (n == 0) return hipSuccess;
  int64_t g = (n + kBlock - 1) / kBlock;
  if (g > 65536) g = 65536;
  hipLaunchKernelGGL(k_fill_zero, dim3(unsigned(g)), dim3(kBlock), 0, s, static_cast<uint32_t*>(p), n);
  return hipGetLastError();
}

hipError_t launch_diag_blocks(const ebe_mesh* m, int level, double* blk6, hipStream_t s) {
  const int64_t n = level == 0 ? m->n_nodes : m->n_vertices;
  hipError_t e = launch_fill_zero(blk6, size_t(n) * 6 * sizeof(double), s);
  if (e != hipSuccess) return e;
  if (level == 0 && m->curved)
    hipLaunchKernelGGL(k_diag_blocks_curved, dim3(grid_for(m->n_elem)), dim3(kBlock), 0, s,
                       m->conn.as<int32_t>(), m->xv.as<double4>(), m->lame64.as<double2>(), blk6, m->n_elem);
  else if (level == 0)
    hipLaunchKernelGGL(k_diag_blocks<0>, dim3(grid_for(m->n_elem)), dim3(kBlock), 0, s,
                       m->conn.as<int32_t>(), m->xv.as<double4>(), m->lame64.as<double2>(), blk6, m->n_elem);
  else
    hipLaunchKernelGGL(k_diag_blocks<1>, dim3(grid_for(m->n_elem)), dim3(kBlock), 0, s,
                       m->conn.as<int32_t>(), m->xv.as<double4>(), m->lame64.as<double2>(), blk6, m->n_elem);
  return hipGetLastError();
}

hipError_t launch_invert_blocks(const ebe_mesh* m, int level, const double* blk6, double* inv64,
                                float* inv32, hipStream_t s) {
  const int64_t n = level_rows(m, level);
  const uint8_t* fx = level == 2 ? m->cfix.as<uint8_t>() : m->fix.as<uint8_t>();
  if (n < 1) return hipSuccess;
  hipLaunchKernelGGL(k_invert_blocks, dim3(grid_for(n)), dim3(kBlock), 0, s, blk6, fx, inv64, inv32, n);
  return hipGetLastError();
}

hipError_t launch_assemble_a2(const ebe_mesh* m, bool assemble, bool f32, hipStream_t s) {
  const int64_t nval = m->a2.slots * 9 * kSliceRows;
  if (assemble) {
    hipLaunchKernelGGL(k_smooth_p2, dim3(grid_for(m->n_vertices)), dim3(kBlock), 0, s, m->k1.soff.as<int32_t>(),
                       m->k1.col.as<int32_t>(), m->k1.val[0].as<double>(), m->fix.as<uint8_t>(),
                       m->agg.as<int32_t>(), m->minv64[1].as<double>(), m->p2_col.as<int32_t>(), m->p2_width,
                       m->p2_val[0].as<double>(), m->p2_val[1].as<float>(), m->n_vertices);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = launch_fill_zero(m->a2.val[0].as<void>(), size_t(nval) * sizeof(double), s);
    if (e != hipSuccess) return e;
    if (m->a2_maxlen > kGalerkinMaxRow) return hipErrorInvalidValue;  // rejected by ensure_level2
    const size_t lds = size_t(m->a2_maxlen) * (9 * sizeof(double) + sizeof(int32_t));
    hipLaunchKernelGGL(k_galerkin_rows, dim3(unsigned(m->n_agg)), dim3(kGalerkinThreads), lds, s,
                       m->k1.soff.as<int32_t>(), m->k1.col.as<int32_t>(), m->k1.val[0].as<double>(),
                       m->fix.as<uint8_t>(), m->p2_col.as<int32_t>(), m->p2_width, m->p2_val[0].as<double>(),
                       m->p2t_off.as<int32_t>(), m->p2t_idx.as<int32_t>(), m->a2.soff.as<int32_t>(),
                       m->a2.col.as<int32_t>(), m->a2_len.as<int32_t>(), m->a2.val[0].as<double>(), m->n_agg);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (!f32 || nval == 0) return hipSuccess;
  int64_t g = (nval + kBlock - 1) / kBlock;
  if (g > 65536) g = 65536;
  hipLaunchKernelGGL(k_to_f32, dim3(unsigned(g)), dim3(kBlock), 0, s, m->a2.val[0].as<double>(),
                     m->a2.val[1].as<float>(), nval);
  return hipGetLastError();
}

hipError_t launch_absmax(const double* a, int64_t n, unsigned long long* out, hipStream_t s) {
  hipError_t e = launch_fill_zero(out, sizeof(unsigned long long), s);
  if (e != hipSuccess || n == 0) return e;
  int64_t g = (n + kBlock - 1) / kBlock;
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(k_absmax, dim3(unsigned(g)), dim3(kBlock), 0, s, a, n, out);
  return hipGetLastError();
}

hipError_t launch_to_f16(const double* a, void* b, int64_t n, double inv_scale, hipStream_t s) {
  if (n == 0) return hipSuccess;
  int64_t g = (n + kBlock - 1) / kBlock;
  if (g > 65536) g = 65536;
  hipLaunchKernelGGL(k_to_f16, dim3(unsigned(g)), dim3(kBlock), 0, s, a, static_cast<_Float16*>(b), n, inv_scale);
  return hipGetLastError();
}

hipError_t launch_asm_diag(const AsmOp& op, double* blk6, hipStream_t s) {
  if (op.rows < 1) return hipSuccess;
  hipLaunchKernelGGL(k_asm_diag, dim3(grid_for(op.rows)), dim3(kBlock), 0, s, op.soff.as<int32_t>(),
                     op.col.as<int32_t>(), op.val[0].as<double>(), blk6, op.rows);
  return hipGetLastError();
}

hipError_t launch_expand_blocks(int64_t n, const double* blk6, double* out9, hipStream_t s) {
  hipLaunchKernelGGL(k_expand_blocks, dim3(grid_for(n)), dim3(kBlock), 0, s, blk6, out9, n);
  return hipGetLastError();
}

hipError_t launch_lame(const ebe_mesh* m, hipStream_t s) {
  hipLaunchKernelGGL(k_lame, dim3(grid_for(m->n_elem)), dim3(kBlock), 0, s, m->young.as<double>(),
                     m->poisson.as<double>(), m->lame64.as<double2>(), m->lame32.as<float2>(), m->n_elem);
  return hipGetLastError();
}

hipError_t launch_geometry(const ebe_mesh* m, ebe_dtype dt, void* out, hipStream_t s) {
  if (dt == EBE_F64)
    hipLaunchKernelGGL(k_geometry<double>, dim3(grid_for(m->n_elem)), dim3(kBlock), 0, s, m->conn.as<int32_t>(),
                       m->xv.as<double4>(), m->lame64.as<double2>(), static_cast<double*>(out), m->n_elem);
  else
    hipLaunchKernelGGL(k_geometry<float>, dim3(grid_for(m->n_elem)), dim3(kBlock), 0, s, m->conn.as<int32_t>(),
                       m->xv.as<double4>(), m->lame64.as<double2>(), static_cast<float*>(out), m->n_elem);
  return hipGetLastError();
}

hipError_t launch_assemble_p1(const ebe_mesh* m, bool assemble, bool f32, hipStream_t s) {
  const int64_t nval = m->k1.slots * 9 * kSliceRows;
  if (assemble) {
    hipLaunchKernelGGL(k_assemble_p1_rows, dim3(grid_for(m->n_vertices)), dim3(kBlock), 0, s,
                       m->conn.as<int32_t>(), m->xv.as<double4>(), m->lame64.as<double2>(),
                       m->v2el_off.as<int32_t>(), m->v2el.as<int32_t>(), m->k1.soff.as<int32_t>(),
                       m->k1.col.as<int32_t>(), m->k1.val[0].as<double>(), m->n_vertices);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (!f32) return hipSuccess;
  int64_t g = (nval + kBlock - 1) / kBlock;
  if (g > 65536) g = 65536;
  hipLaunchKernelGGL(k_to_f32, dim3(unsigned(g < 1 ? 1 : g)), dim3(kBlock), 0, s, m->k1.val[0].as<double>(),
                     m->k1.val[1].as<float>(), nval);
  return hipGetLastError();
}

hipError_t launch_check_material(const double* young, const double* poisson, int64_t n, int* bad,
                                 hipStream_t s) {
  hipError_t e = launch_fill_zero(bad, sizeof(int), s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_check_material, dim3(grid_for(n)), dim3(kBlock), 0, s, young, poisson, bad, n);
  return hipGetLastError();
}

}  // namespace ebe
