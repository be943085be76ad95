// Element-by-element products on gfx950 (Section 2, Eq. (3)): y = K x for the
// quadratic mesh and y = K1 x for the linear (corner) mesh, n cases at once.
//
// Work decomposition (see patches.cpp).  One workgroup per element patch
// (quadratic level: <= 64 elements, <= 192 nodes; linear level: <= 256
// elements, <= 128 corners):
//   1. one work-item per element puts the element geometry (gradients,
//      volume, Lame constants: from the four corner coordinates and the
//      material, or from the mesh's cache of exactly those values) into LDS;
//      the element matrix itself is never stored but rebuilt from it at
//      every product (Section 2);
//   2. one work-item per (element, case) streams the element's nodal values
//      through K_e (p2_element.h) and adds each nodal force into an FP64 LDS
//      accumulator F[node][component][case] (FP32 LDS atomics are much slower
//      on this part).  The nodal values come in one of two forms:
//        gather: straight from x (the n cases of a node are contiguous:
//          Section 3.1's case loop), all cases in one pass;
//        staged: the cases are taken in passes of at most 8 (FP32: two
//          workgroups per CU) or 8 (FP64, 1024 work-items); a pass first
//          copies the patch's node rows into LDS with coalesced vector loads;
//      which form is faster depends on the dtype, n and the mesh, and is
//      measured per mesh (autotune.cpp);
//   3. each patch node is written once per pass: exclusive nodes straight
//      into y, shared nodes as a partial sum into their staging slot.
// A second, node-centric kernel adds the consecutive staged partials of each
// shared node in patch order.  Global memory sees no atomics, every node is
// written exactly once per product (so y needs no clearing pass), and the
// result does not depend on scheduling.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <type_traits>

#include "ebe_internal.h"
#include "p2_element.h"
#include "patch_common.h"

namespace ebe {
namespace {

// STAGE: the staged form (else the gather form).  CURVED: isoparametric
// quadratic elements (quadratic level, gather form): phase 1 forms each
// element's four quadrature-point gradients and weights from its ten node
// coordinates (xv then holds every node), phase 2 applies p2c_apply.  MASK: zero the fixed
// DOFs of x while reading it (y = P K P x); callers whose x is already zero
// there (the solver) skip it, and the kernel then has no masking code.  bc: zero the fixed DOFs of y.  add: y += K x
// instead of y = K x.  gamma (optional): gamma[r] += (x_r, K x_r) formed
// element by element as sum_e x_eᵀ K_e x_e, which is what CG needs from
// q = K p without a separate inner-product pass.
template <typename T, int NR, int ORDER, bool STAGE, bool MASK, bool CURVED>
__global__ __launch_bounds__(threads_for(NR, ORDER, int(sizeof(T)), STAGE))
__attribute__((amdgpu_waves_per_eu(patch_waves_per_simd<T>(NR, ORDER, STAGE, CURVED)))) void k_ebe_patch(
    const int32_t* __restrict__ conn, const uint8_t* __restrict__ lconn, const int32_t* __restrict__ pelem,
    const int32_t* __restrict__ poff, const int32_t* __restrict__ pnode, const int32_t* __restrict__ pslot,
    const double4* __restrict__ xv, const typename Pair<T>::type* __restrict__ lame, const T* __restrict__ x,
    T* __restrict__ y, T* __restrict__ stage, int stream, int bc, int add, double* __restrict__ gamma,
    double* __restrict__ gslot, unsigned* __restrict__ gcount, const int* __restrict__ gate,
    const T* __restrict__ gcache) {
  constexpr int NLOC = ORDER == 2 ? 10 : 4;
  constexpr int CW = chunk_for(NR, ORDER, int(sizeof(T)), STAGE);  // cases per pass
  constexpr int NPASS = (NR + CW - 1) / CW;
  constexpr int W = 3 * NR;   // values of a node in x, y and the staging buffer
  constexpr int WC = 3 * CW;  // values of a node in one pass
  constexpr int TPB = threads_for(NR, ORDER, int(sizeof(T)), STAGE);
  constexpr int MAXN = ORDER == 2 ? kPatchNodes : kLinPatchCorners;
  constexpr int PE = ORDER == 2 ? kPatchElems : kLinPatchElems;
  constexpr int VEC = pass_vec(NR, CW, int(sizeof(T)));  // values per vector access of a node row
  constexpr int NV = WC / VEC;                            // vectors of a node in one pass
  // Node-row staging: work-item t moves vector t % NV of nodes t / NV,
  // t / NV + EPK, ... (EPK = TPB / NV nodes per sweep), so its place in the
  // row, and with it the case and component, never changes.
  constexpr int EPK = TPB / NV;                           // nodes per sweep
  constexpr int KIT = (MAXN + EPK - 1) / EPK;             // sweeps per pass, at most
  using V = VecT<T, VEC>;
  __shared__ double F[MAXN * WC];
  __shared__ __align__(16) T X[STAGE ? MAXN * WC : 1];
  static_assert(!CURVED || (ORDER == 2 && !STAGE), "curved elements: quadratic level, gather form");
  // element data: straight, G (12), lambda V s, mu V s; curved, per
  // quadrature point q at 12 q: grad L_1..L_3 (9), lambda det J / 24, mu det J / 24
  __shared__ __align__(16) T geo[PE][CURVED ? 48 : 14];
  __shared__ int32_t words[MAXN];
  __shared__ int32_t slots[MAXN];
  __shared__ double gsum[NR];
  if (gate && *gate == 0) return;
  const int tid = threadIdx.x;
  const int p = xcd_patch(blockIdx.x, gridDim.x);
  const int e0 = pelem[p], ne = pelem[p + 1] - e0;
  const int o0 = poff[p], nn = poff[p + 1] - o0;
  for (int i = tid; i < nn; i += TPB) {
    words[i] = pnode[o0 + i];
    slots[i] = pslot[o0 + i];
  }
  if (tid < NR) gsum[tid] = 0.0;
  if constexpr (CURVED) {
    for (int w = tid; w < 4 * ne; w += TPB) {
      const int el = w >> 2, q = w & 3;
      const int64_t e = int64_t(e0) + el;
      const double4 x0 = xv[conn[e * 10] & kIdxMask];
      double d[10][3];
#pragma unroll
      for (int a = 0; a < 10; ++a) {
        const double4 xa = xv[conn[e * 10 + a] & kIdxMask];
        d[a][0] = xa.x - x0.x;
        d[a][1] = xa.y - x0.y;
        d[a][2] = xa.z - x0.z;
      }
      double G[3][3];
      const double wdet = curved_point(d, q, G) * (1.0 / 24.0);
      T* g = &geo[el][12 * q];
#pragma unroll
      for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int dd = 0; dd < 3; ++dd) g[3 * j + dd] = T(G[j][dd]);
      const auto lm = lame[e];
      g[9] = T(double(lm.x) * wdet);
      g[10] = T(double(lm.y) * wdet);
    }
  }
  for (int el = tid; el < (CURVED ? 0 : ne); el += TPB) {
    const int64_t e = int64_t(e0) + el;
    if (gcache) {  // the mesh's geometry cache: one row per element, formed exactly as below
      const T* g = gcache + e * 16;
#pragma unroll
      for (int i = 0; i < 12; ++i) geo[el][i] = g[i];
      const T sv = ORDER == 2 ? g[12] * T(0.05) : g[12];
      geo[el][12] = g[13] * sv;
      geo[el][13] = g[14] * sv;
      continue;
    }
    store_geometry<T, ORDER>(geo[el], xv[conn[e * 10 + 0] & kIdxMask], xv[conn[e * 10 + 1] & kIdxMask],
                             xv[conn[e * 10 + 2] & kIdxMask], xv[conn[e * 10 + 3] & kIdxMask], lame[e]);
  }
  // (x, K x) contributions: when the pass width divides 64 a work-item keeps
  // one case for all its items, so it sums them in a register and the lanes
  // of a case are combined across the wavefront before one LDS atomic.
  constexpr bool kLaneCase = (64 % CW) == 0 && (TPB % CW) == 0;
  const int nj = spread_count<CW>(ne);
  const int sv = tid % NV;                 // this work-item's vector in a node row
  const int sent = tid < EPK * NV ? tid / NV : MAXN;  // its first node (none if past the sweep)
  const int sq = sv * VEC;                 // value offset in the pass row
  const int sc = sq / CW, scc = sq - sc * CW;  // component and first case of the vector
  __syncthreads();
#pragma unroll 1
  for (int pass = 0; pass < NPASS; ++pass) {
    const int c0 = pass * CW;
    const int cw = NR - c0 < CW ? NR - c0 : CW;
    // Clear the accumulator and (staged form) copy this pass's node rows,
    // zero for fixed DOFs under mask_in and for the unused lanes of a short
    // last pass.  A fixed trip count lets every work-item issue all its loads
    // at once.
#pragma unroll
    for (int k = 0; k < KIT; ++k) {
      const int ent = sent + k * EPK;
      if (ent < nn) {
        const int q = sq, c = sc, cc = scc;
        if constexpr (STAGE) {
          const int32_t wd = words[ent];
          V v;
          if (cc < cw && !(MASK && ((wd >> (kIdxBits + c)) & 1))) {
            v = *reinterpret_cast<const V*>(x + size_t(uint32_t(wd) & uint32_t(kIdxMask)) * W + c * NR + c0 + cc);
          } else {
#pragma unroll
            for (int t = 0; t < VEC; ++t) v.v[t] = T(0);
          }
          *reinterpret_cast<V*>(X + ent * WC + q) = v;
        }
#pragma unroll
        for (int t = 0; t < VEC; ++t) F[ent * WC + q + t] = 0.0;
      }
    }
    __syncthreads();
    double en_acc = 0.0;
    for (int w = tid; w < nj * CW; w += TPB) {
      const int j = w / CW;
      const int r = w - j * CW;
      const int el = spread_element<CW>(j, ne);
      if (el >= ne || r >= cw) continue;
      const int64_t e = int64_t(e0) + el;
      int lid[NLOC];  // F (and X) index of the node's first component in this work-item's case
      int gw[NLOC];   // gather form: the node's word (id and Dirichlet bits)
      if constexpr (ORDER == 2) {
        const uint4 q = *reinterpret_cast<const uint4*>(lconn + e * 16);
        const uint32_t qw[3] = {q.x, q.y, q.z};
#pragma unroll
        for (int a = 0; a < NLOC; ++a) lid[a] = (qw[a >> 2] >> (8 * (a & 3))) & 0xff;
      } else {
        const uint32_t q = *reinterpret_cast<const uint32_t*>(lconn + e * 4);
#pragma unroll
        for (int a = 0; a < NLOC; ++a) lid[a] = (q >> (8 * a)) & 0xff;
      }
#pragma unroll
      for (int a = 0; a < NLOC; ++a) {
        if constexpr (!STAGE) gw[a] = words[lid[a]];
        lid[a] = lid[a] * WC + r;
      }
      T en = T(0);
      auto u = [&](int a, int c) -> T {
        if constexpr (STAGE) {
          return X[lid[a] + c * CW];
        } else {
          const T v = x[size_t(uint32_t(gw[a]) & uint32_t(kIdxMask)) * W + c * NR + r];
          return (MASK && ((gw[a] >> (kIdxBits + c)) & 1)) ? T(0) : v;
        }
      };
      auto emit = [&](int a, const T f[3]) {
#pragma unroll
        for (int c = 0; c < 3; ++c) atomicAdd(F + lid[a] + c * CW, double(f[c]));
      };
      if constexpr (CURVED) {
        const T* gr = geo[el];
        p2c_apply<T>([&](int q, int i) { return gr[12 * q + i]; }, u, emit, gamma != nullptr, en);
      } else {
        T G[4][3];
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
          for (int d = 0; d < 3; ++d) G[k][d] = geo[el][3 * k + d];
        const T cl = geo[el][12], cm = geo[el][13];
        if constexpr (ORDER == 2) p2_apply<T>(G, cl, cm, u, emit, gamma != nullptr, en);
        else p1_apply<T>(G, cl, cm, u, emit, gamma != nullptr, en);
      }
      if (gamma) {
        if constexpr (kLaneCase) en_acc += double(en);
        else atomicAdd(&gsum[c0 + r], double(en));
      }
    }
    if constexpr (kLaneCase) {
      if (gamma) {
#pragma unroll
        for (int off = 32; off >= CW; off >>= 1) en_acc += __shfl_xor(en_acc, off, 64);
        if ((tid & 63) < cw) atomicAdd(&gsum[c0 + (tid & 63)], en_acc);
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < KIT; ++k) {
      const int ent = sent + k * EPK;
      if (ent < nn) {
        const int q = sq, c = sc, cc = scc;
        if (cc < cw) {
          const int32_t wd = words[ent];
          const int col = c * NR + c0 + cc;
          V v;
#pragma unroll
          for (int t = 0; t < VEC; ++t) v.v[t] = T(F[ent * WC + q + t]);
          if (wd < 0) {  // shared node: partial sum to its staging slot
            T* sp = stage + size_t(slots[ent]) * W + col;
          if (stream) store_stream<T, VEC>(sp, v);
          else *reinterpret_cast<V*>(sp) = v;
          } else {
            V* yp = reinterpret_cast<V*>(y + size_t(wd & kIdxMask) * W + col);
            const bool fixed = bc && ((wd >> (kIdxBits + c)) & 1);
            if (add) {
              if (!fixed) {
                V o = *yp;
#pragma unroll
                for (int t = 0; t < VEC; ++t) o.v[t] += v.v[t];
                *yp = o;
              }
            } else {
              if (fixed) {
#pragma unroll
                for (int t = 0; t < VEC; ++t) v.v[t] = T(0);
              }
              *yp = v;
            }
          }
        }
      }
    }
    if (pass + 1 < NPASS) __syncthreads();  // X and F are refilled by the next pass
  }
  if (gamma) fold_gamma<NR, TPB>(gsum, gamma, gslot, gcount);
}

// Assembled linear-level form: y = K1 x with the 3x3 blocks of K1 in slices
// of kSliceRows rows (slot j of row r at entry j * kSliceRows + r, values
// value-major within the slot, so the rows of a wavefront read each value
// and column word from one contiguous run).  A work-item forms the three
// rows of block row v for CPL consecutive cases (NR / CPL work-items per
// row, RPB rows per workgroup, rows grid-strided): a block value it reads
// serves CPL cases and its x reads are whole vectors.  mask_in, bc, add and
// gamma as in the patch forms; gamma takes (x_v, (K x)_v) before the
// projection of y.
#ifndef EBE_ASM_CPL_F32
#define EBE_ASM_CPL_F32 4
#endif
#ifndef EBE_ASM_CPL_F64
#define EBE_ASM_CPL_F64 4
#endif
#ifndef EBE_ASM_UNROLL_F32
#define EBE_ASM_UNROLL_F32 4
#endif
#ifndef EBE_ASM_UNROLL_F64
#define EBE_ASM_UNROLL_F64 1
#endif
#ifndef EBE_ASM_WG_PER_CU
#define EBE_ASM_WG_PER_CU 8
#endif
// Tiles of the assembled product (cases per work-item, slots per trip), one
// per kernel variant: 0 is the default, 1 and 2 are in the tuner's search.
constexpr int asm_tile_cpl(bool f32, int v) {
  return f32 ? (v == 1 ? 2 : (v == 2 ? 8 : EBE_ASM_CPL_F32)) : (v == 1 ? 2 : (v == 2 ? 1 : EBE_ASM_CPL_F64));
}
constexpr int asm_tile_unroll(bool f32, int v) {
  return f32 ? (v == 1 ? 4 : (v == 2 ? 2 : EBE_ASM_UNROLL_F32)) : (v == 1 ? 2 : (v == 2 ? 4 : EBE_ASM_UNROLL_F64));
}
template <typename T, int NR, int V = 0>
constexpr int asm_cpl() {
  int c = asm_tile_cpl(sizeof(T) == 4, V);
  while (c > 1 && NR % c != 0) c /= 2;
  return c;
}
template <typename T, int NR, int V = 0>
constexpr int asm_rows() { return 256 / (NR / asm_cpl<T, NR, V>()); }
template <typename T, int NR, int V = 0>
constexpr int asm_threads() { return asm_rows<T, NR, V>() * (NR / asm_cpl<T, NR, V>()); }

// S: the stored value type (T, or FP16 holding the values divided by vscale,
// which multiplies each row's sums at the end).  TV: the tile variant.
template <typename T, int NR, typename S = T, int TV = 0>
__global__ __launch_bounds__((asm_threads<T, NR, TV>())) void k_assembled(
    const int32_t* __restrict__ soff, const int32_t* __restrict__ col, const S* __restrict__ val,
    const uint8_t* __restrict__ fix, const T* __restrict__ x, T* __restrict__ y, int64_t nv, int mask_in, int bc,
    int add, double* __restrict__ gamma, double* __restrict__ gslot, unsigned* __restrict__ gcount,
    const int* __restrict__ gate, T vscale = T(1)) {
  constexpr int W = 3 * NR;
  constexpr int CPL = asm_cpl<T, NR, TV>();
  constexpr int LPR = NR / CPL;  // work-items per row
  constexpr int RPB = asm_rows<T, NR, TV>();
  constexpr int VW = CPL * int(sizeof(T)) > 16 ? 16 / int(sizeof(T)) : CPL;  // values per (<= 16-byte) vector
  constexpr int NVEC = CPL / VW;
  constexpr int SR = kSliceRows;
  constexpr int U = asm_tile_unroll(sizeof(T) == 4, TV);  // slots per trip
  using V = VecT<T, VW>;
  __shared__ double gsum[NR];
  if (gate && *gate == 0) return;
  const int tid = threadIdx.x;
  if (gamma) {
    if (tid < NR) gsum[tid] = 0.0;
    __syncthreads();
  }
  const int lr = tid / LPR;
  const int j0 = (tid - lr * LPR) * CPL;
  double en[CPL];
#pragma unroll
  for (int t = 0; t < CPL; ++t) en[t] = 0.0;
  // chunks of RPB rows: XCD x owns a contiguous chunk range (so the x rows a
  // chunk's neighbours share are read through one L2); its g-th workgroup
  // takes start + g, start + g + wx, ...  Every XCD has a workgroup whenever
  // the range is not empty (the grid is at least 8, or one per chunk).
  const int64_t nch = (nv + RPB - 1) / RPB;
  const int xcd = int(blockIdx.x) % kXcds;
  const int64_t wx = (int64_t(gridDim.x) - xcd + kXcds - 1) / kXcds;
  const int64_t cq = nch / kXcds, cr = nch % kXcds;
  const int64_t stop = xcd * cq + (xcd < cr ? xcd : cr) + cq + (xcd < cr ? 1 : 0);
  for (int64_t ch = stop - cq - (xcd < cr ? 1 : 0) + int64_t(blockIdx.x) / kXcds; ch < stop; ch += wx) {
    const int64_t v = ch * RPB + lr;
    if (v >= nv) continue;
    const int64_t sl = v / SR;
    const int r = int(v - sl * SR);
    T acc[3][CPL];
#pragma unroll
    for (int q = 0; q < 3; ++q)
#pragma unroll
      for (int t = 0; t < CPL; ++t) acc[q][t] = T(0);
    // U slots per trip, their column words loaded one trip ahead, so a trip
    // waits for one round of loads (x rows and values) instead of two.  Slot
    // indices past the row are clamped to its last slot (always present: the
    // diagonal) and their blocks skipped.
    const int32_t kb = soff[sl], k1 = soff[sl + 1];
    const int32_t* cp = col + r;
    int32_t wn[U];
#pragma unroll
    for (int u = 0; u < U; ++u) wn[u] = cp[size_t(min(kb + u, k1 - 1)) * SR];
    for (int32_t k = kb; k < k1; k += U) {
      int32_t w[U];
#pragma unroll
      for (int u = 0; u < U; ++u) w[u] = wn[u];
      if (k + U < k1) {
#pragma unroll
        for (int u = 0; u < U; ++u) wn[u] = cp[size_t(min(k + U + u, k1 - 1)) * SR];
      }
      T xc[U][3][CPL];
      T b[U][9];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const T* xp = x + size_t(uint32_t(w[u]) & uint32_t(kIdxMask)) * W + j0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
#pragma unroll
          for (int q = 0; q < NVEC; ++q) {
            const V xv = *reinterpret_cast<const V*>(xp + c * NR + q * VW);
#pragma unroll
            for (int t = 0; t < VW; ++t) xc[u][c][q * VW + t] = xv.v[t];
          }
        }
        const S* a = val + size_t(min(k + u, k1 - 1)) * 9 * kSliceRows + r;
#pragma unroll
        for (int i = 0; i < 9; ++i) b[u][i] = T(a[i * kSliceRows]);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (k + u >= k1) break;
#pragma unroll
        for (int c = 0; c < 3; ++c)
          if (mask_in && ((w[u] >> (kIdxBits + c)) & 1)) {
#pragma unroll
            for (int t = 0; t < CPL; ++t) xc[u][c][t] = T(0);
          }
#pragma unroll
        for (int q = 0; q < 3; ++q)
#pragma unroll
          for (int t = 0; t < CPL; ++t)
            acc[q][t] += b[u][3 * q] * xc[u][0][t] + b[u][3 * q + 1] * xc[u][1][t] + b[u][3 * q + 2] * xc[u][2][t];
      }
    }
    if constexpr (!std::is_same<S, T>::value) {
#pragma unroll
      for (int q = 0; q < 3; ++q)
#pragma unroll
        for (int t = 0; t < CPL; ++t) acc[q][t] *= vscale;
    }
    const int fb = fix[v];
    if (gamma) {
      const T* xo = x + size_t(v) * W + j0;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const bool zero = mask_in && ((fb >> c) & 1);
#pragma unroll
        for (int q = 0; q < NVEC; ++q) {
          const V xv = *reinterpret_cast<const V*>(xo + c * NR + q * VW);
#pragma unroll
          for (int t = 0; t < VW; ++t) en[q * VW + t] += zero ? 0.0 : double(xv.v[t]) * double(acc[c][q * VW + t]);
        }
      }
    }
    T* yp = y + size_t(v) * W + j0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const bool fixed = bc && ((fb >> c) & 1);
#pragma unroll
      for (int q = 0; q < NVEC; ++q) {
        V* vp = reinterpret_cast<V*>(yp + c * NR + q * VW);
        V o;
        if (add) {
          o = *vp;
          if (!fixed) {
#pragma unroll
            for (int t = 0; t < VW; ++t) o.v[t] += acc[c][q * VW + t];
          }
        } else {
#pragma unroll
          for (int t = 0; t < VW; ++t) o.v[t] = fixed ? T(0) : acc[c][q * VW + t];
        }
        *vp = o;
      }
    }
  }
  if (gamma) {
#pragma unroll
    for (int t = 0; t < CPL; ++t) atomicAdd(&gsum[j0 + t], en[t]);
    __syncthreads();
    fold_gamma<NR, (asm_threads<T, NR, TV>())>(gsum, gamma, gslot, gcount);
  }
}

// cache: read the element geometry from the mesh's cache (when it is filled),
// else form it from the corner coordinates in the kernel
template <typename T, int NR, int ORDER, bool STAGE, bool MASK, bool CURVED = false>
void launch_patch_m(const ebe_mesh* m, const PatchLevel& L, const void* x, void* y, T* stage, bool stream, bool bc,
                    bool add, const int* gate, hipStream_t s, double* gamma, bool cache = true) {
  using P = typename Pair<T>::type;
  const P* lame = (sizeof(T) == 8) ? reinterpret_cast<const P*>(m->lame64.as<void>())
                                   : reinterpret_cast<const P*>(m->lame32.as<void>());
  hipLaunchKernelGGL((k_ebe_patch<T, NR, ORDER, STAGE, MASK, CURVED>), dim3(unsigned(L.npatch)),
                     dim3(threads_for(NR, ORDER, int(sizeof(T)), STAGE)), 0, s, m->conn.as<int32_t>(),
                     ORDER == 2 ? m->lconn.as<uint8_t>() : m->lconn1.as<uint8_t>(), L.pelem.as<int32_t>(),
                     L.poff.as<int32_t>(), L.pnode.as<int32_t>(), L.pslot.as<int32_t>(), m->xv.as<double4>(), lame,
                     static_cast<const T*>(x), static_cast<T*>(y), stage, int(stream), int(bc), int(add), gamma,
                     m->gacc.as<double>(), reinterpret_cast<unsigned*>(m->gacc.as<char>() + kGammaBytes - 64),
                     gate,
                     !CURVED && cache && m->geo_ready[sizeof(T) == 8 ? 0 : 1] ? m->geo[sizeof(T) == 8 ? 0 : 1].as<T>()
                                                                              : nullptr);
}

template <typename T, int NR, int ORDER, bool STAGE, bool CURVED = false>
void launch_patch(const ebe_mesh* m, const PatchLevel& L, const void* x, void* y, T* stage, bool stream,
                  bool mask_in, bool bc, bool add, const int* gate, hipStream_t s, double* gamma, bool cache = true) {
  if (mask_in)
    launch_patch_m<T, NR, ORDER, STAGE, true, CURVED>(m, L, x, y, stage, stream, bc, add, gate, s, gamma, cache);
  else
    launch_patch_m<T, NR, ORDER, STAGE, false, CURVED>(m, L, x, y, stage, stream, bc, add, gate, s, gamma, cache);
}
// y = A x for an assembled operator whose row fix bits are `fix`
template <typename T, int NR, int V = 0>
hipError_t launch_asm_p(const ebe_mesh* m, const AsmOp& op, const uint8_t* fix, const void* x, void* y,
                        bool mask_in, bool bc, bool add, const int* gate, hipStream_t s, double* gamma) {
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, m->device) != hipSuccess || cus < 1)
    cus = 256;
  constexpr int RPB = asm_rows<T, NR, V>();
  const int64_t grid =
      std::max<int64_t>(1, std::min<int64_t>((op.rows + RPB - 1) / RPB, int64_t(EBE_ASM_WG_PER_CU) * cus));
  hipLaunchKernelGGL((k_assembled<T, NR, T, V>), dim3(unsigned(grid)), dim3(asm_threads<T, NR, V>()), 0, s,
                     op.soff.as<int32_t>(), op.col.as<int32_t>(), op.val[sizeof(T) == 8 ? 0 : 1].as<T>(), fix,
                     static_cast<const T*>(x), static_cast<T*>(y), op.rows, int(mask_in), int(bc), int(add), gamma,
                     m->gacc.as<double>(), reinterpret_cast<unsigned*>(m->gacc.as<char>() + kGammaBytes - 64),
                     gate);
  return hipGetLastError();
}

template <int NR>
hipError_t launch_asm_half_p(const ebe_mesh* m, const AsmOp& op, const uint8_t* fix, const float* x, float* y,
                             bool mask_in, bool bc, bool add, const int* gate, hipStream_t s, double* gamma) {
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, m->device) != hipSuccess || cus < 1)
    cus = 256;
  constexpr int RPB = asm_rows<float, NR>();
  const int64_t grid =
      std::max<int64_t>(1, std::min<int64_t>((op.rows + RPB - 1) / RPB, int64_t(EBE_ASM_WG_PER_CU) * cus));
  hipLaunchKernelGGL((k_assembled<float, NR, _Float16>), dim3(unsigned(grid)), dim3(asm_threads<float, NR>()), 0, s,
                     op.soff.as<int32_t>(), op.col.as<int32_t>(), op.val16.as<_Float16>(), fix, x, y, op.rows,
                     int(mask_in), int(bc), int(add), gamma, m->gacc.as<double>(),
                     reinterpret_cast<unsigned*>(m->gacc.as<char>() + kGammaBytes - 64), gate, float(op.half_scale));
  return hipGetLastError();
}

template <typename T, int NR>
hipError_t ebe_dispatch_p(int order, int form, const ebe_mesh* m, const void* x, void* y, bool mask_in, bool bc,
                          bool add, const int* gate, hipStream_t s, double* gamma) {
  const PatchLevel& L = m->pl[order == 2 ? 0 : 1];
  T* stage = L.stage.as<T>();
  if (form == EBE_FORM_ASSEMBLED) {  // linear level only (checked by the caller); tile variant 0..2
    const int var = m->fvar[1][sizeof(T) == 8 ? 0 : 1][NR];
    const uint8_t* fx = m->fix.as<uint8_t>();
    if (var == 1) return launch_asm_p<T, NR, 1>(m, m->k1, fx, x, y, mask_in, bc, add, gate, s, gamma);
    if (var == 2) return launch_asm_p<T, NR, 2>(m, m->k1, fx, x, y, mask_in, bc, add, gate, s, gamma);
    return launch_asm_p<T, NR>(m, m->k1, fx, x, y, mask_in, bc, add, gate, s, gamma);
  }
  if (form == EBE_FORM_PIPELINED || form == EBE_FORM_COLOURED) {
    const bool colour = form == EBE_FORM_COLOURED;
    const int var = m->fvar[order == 2 ? 0 : 1][sizeof(T) == 8 ? 0 : 1][NR];
    if (order == 2)
      return var != 1 ? launch_pipe<T, NR, 2, true, 1>(m, x, y, mask_in, bc, add, gate, s, gamma, colour)
                      : launch_pipe<T, NR, 2, false, 1>(m, x, y, mask_in, bc, add, gate, s, gamma, colour);
    return var != 1 ? launch_pipe<T, NR, 1, true, 1>(m, x, y, mask_in, bc, add, gate, s, gamma, colour)
                    : launch_pipe<T, NR, 1, false, 1>(m, x, y, mask_in, bc, add, gate, s, gamma, colour);
  }
  // stream the staged partials past the caches when they cannot stay in the
  // last-level cache until the shared-node pass reads them back
  const bool st = int64_t(L.nslots) * 3 * NR * int64_t(sizeof(T)) > kStreamStageBytes;
  // variant 1: element geometry formed from the corner coordinates (less
  // memory traffic than the cache rows where few cases share an element)
  const bool cache = m->fvar[order == 2 ? 0 : 1][sizeof(T) == 8 ? 0 : 1][NR] != 1;
  if (order == 2 && m->curved) {  // gather form only (form_usable)
    launch_patch<T, NR, 2, false, true>(m, L, x, y, stage, st, mask_in, bc, add, gate, s, gamma);
  } else if (order == 2) {
    if (form == EBE_FORM_STAGED)
      launch_patch<T, NR, 2, true>(m, L, x, y, stage, st, mask_in, bc, add, gate, s, gamma, cache);
    else
      launch_patch<T, NR, 2, false>(m, L, x, y, stage, st, mask_in, bc, add, gate, s, gamma, cache);
  } else {
    if (form == EBE_FORM_STAGED)
      launch_patch<T, NR, 1, true>(m, L, x, y, stage, st, mask_in, bc, add, gate, s, gamma, cache);
    else
      launch_patch<T, NR, 1, false>(m, L, x, y, stage, st, mask_in, bc, add, gate, s, gamma, cache);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || L.nshared == 0) return e;
  const int64_t work = L.nshared * (3 * NR / reduce_width<T, NR>());
  hipLaunchKernelGGL((k_reduce_shared<T, NR>), dim3(unsigned((work + 255) / 256)), dim3(256), 0, s,
                     L.snode.as<int32_t>(), L.soff.as<int32_t>(), stage, int(st), static_cast<T*>(y), int32_t(L.nshared),
                     int(bc), int(add), gate);
  return hipGetLastError();
}

template <typename T>
hipError_t ebe_dispatch(int order, int form, const ebe_mesh* m, int nrhs, const void* x, void* y, bool mask_in,
                        bool bc, bool add, const int* gate, hipStream_t s, double* gamma) {
  switch (nrhs) {
#define EBE_CASE(n) \
  case n: return ebe_dispatch_p<T, n>(order, form, m, x, y, mask_in, bc, add, gate, s, gamma);
    EBE_CASE(1) EBE_CASE(2) EBE_CASE(3) EBE_CASE(4) EBE_CASE(5) EBE_CASE(6) EBE_CASE(7) EBE_CASE(8)
    EBE_CASE(9) EBE_CASE(10) EBE_CASE(11) EBE_CASE(12) EBE_CASE(13) EBE_CASE(14) EBE_CASE(15) EBE_CASE(16)
#undef EBE_CASE
    default: return hipErrorInvalidValue;
  }
}

// ---- allocation-free product -------------------------------------------
// Staging memory of ebe_matvec_noalloc: a fixed array in the code object, so
// that the call needs no device allocation.  Each device the library runs on
// holds its own copy until the process ends.  Host code never passes the
// array's name to a kernel (on the host it is only a stand-in for the
// symbol): the device address comes from hipGetSymbolAddress, looked up once
// per device with that device current, and kept below.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void* scratch_dev[kMaxDevices] = {};

template <typename T, int NR>
hipError_t launch_noalloc_p(const ebe_mesh* m, const void* x, void* y, bool bc, void* stage, hipStream_t s) {
  const PatchLevel& L = m->pl[0];
  T* st = static_cast<T*>(stage);
  if (m->curved) {
    if (bc) launch_patch_m<T, NR, 2, false, true, true>(m, L, x, y, st, false, bc, false, nullptr, s, nullptr);
    else launch_patch_m<T, NR, 2, false, false, true>(m, L, x, y, st, false, bc, false, nullptr, s, nullptr);
  } else {
    if (bc) launch_patch_m<T, NR, 2, false, true>(m, L, x, y, st, false, bc, false, nullptr, s, nullptr);
    else launch_patch_m<T, NR, 2, false, false>(m, L, x, y, st, false, bc, false, nullptr, s, nullptr);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || L.nshared == 0) return e;
  const int64_t work = L.nshared * (3 * NR / reduce_width<T, NR>());
  hipLaunchKernelGGL((k_reduce_shared<T, NR>), dim3(unsigned((work + 255) / 256)), dim3(256), 0, s,
                     L.snode.as<int32_t>(), L.soff.as<int32_t>(), st, 0, static_cast<T*>(y), int32_t(L.nshared),
                     int(bc), 0, nullptr);
  return hipGetLastError();
}

}  // namespace

ebe_status noalloc_scratch(int device, void** ptr) {
  if (device < 0 || device >= kMaxDevices) {
    set_error("no-allocation scratch: device %d outside 0..%d", device, kMaxDevices - 1);
    return EBE_ERR_ARG;
  }
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_dev[device]) {
    int prev = 0;
    EBE_TRY_HIP(hipGetDevice(&prev));
    EBE_TRY_HIP(hipSetDevice(device));
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    (void)hipSetDevice(prev);
    if (e != hipSuccess || !p) {
      set_error("hipGetSymbolAddress(scratch) on device %d failed: %s", device, hipGetErrorString(e));
      return EBE_ERR_HIP;
    }
    scratch_dev[device] = p;
  }
  *ptr = scratch_dev[device];
  return EBE_OK;
}

hipError_t launch_ebe_noalloc(const ebe_mesh* m, ebe_dtype dt, int nrhs, const void* x, void* y, bool bc,
                              void* stage, hipStream_t s) {
  if (nrhs < 1 || nrhs > EBE_MAX_RHS || m->pl[0].npatch < 1 ||
      size_t(m->pl[0].nslots) * 3 * size_t(nrhs) * (dt == EBE_F64 ? 8 : 4) > kNoAllocScratchBytes)
    return hipErrorInvalidValue;  // checked by the entry point: host bug
  switch (nrhs) {
#define EBE_CASE(n)                                                              \
  case n:                                                                        \
    return dt == EBE_F64 ? launch_noalloc_p<double, n>(m, x, y, bc, stage, s)    \
                         : launch_noalloc_p<float, n>(m, x, y, bc, stage, s);
    EBE_CASE(1) EBE_CASE(2) EBE_CASE(3) EBE_CASE(4) EBE_CASE(5) EBE_CASE(6) EBE_CASE(7) EBE_CASE(8)
    EBE_CASE(9) EBE_CASE(10) EBE_CASE(11) EBE_CASE(12) EBE_CASE(13) EBE_CASE(14) EBE_CASE(15) EBE_CASE(16)
#undef EBE_CASE
    default: return hipErrorInvalidValue;
  }
}

ebe_status ensure_stage(ebe_mesh* m, int nrhs, size_t elem_bytes) {
  for (int l = 0; l < 2; ++l) {
    const PatchLevel& L = m->pl[l];
    if ((L.nslots + 1) * 3 * EBE_MAX_RHS >= (int64_t(1) << 31) ||
        (L.nshared + 1) * 3 * EBE_MAX_RHS >= (int64_t(1) << 31)) {
      set_error("mesh too large for 32-bit staging indices (%lld slots)", (long long)L.nslots);
      return EBE_ERR_ARG;
    }
    const size_t need = size_t(L.nslots) * 3 * size_t(nrhs) * elem_bytes;
    ebe_status st = m->pl[l].stage.alloc(need);
    if (st != EBE_OK) return st;
  }
  return EBE_OK;
}

bool form_available(int order, int form) {
  return form >= 0 && form < EBE_NUM_FORMS && (form != EBE_FORM_ASSEMBLED || order == 1) &&
         ((form != EBE_FORM_COLOURED && form != EBE_FORM_DETERMINISTIC) || order == 2);
}

bool form_usable(const ebe_mesh* m, int order, int form, ebe_dtype dt, int nrhs) {
  if (!form_available(order, form)) return false;
  if (order == 2 && m->curved) return form == EBE_FORM_GATHER;  // the curved element kernel
  if (form == EBE_FORM_DETERMINISTIC) return m->pl[0].pinc.bytes() > 0;
  if (form != EBE_FORM_PIPELINED && form != EBE_FORM_COLOURED) return true;
  const PatchLevel& L = m->pl[order == 2 ? 0 : 1];
  // node tables hold 32-bit byte offsets of node rows
  const int64_t rows = order == 2 ? m->n_nodes : m->n_vertices;
  const int64_t row_bytes = int64_t(3) * nrhs * (dt == EBE_F64 ? 8 : 4);
  if (L.ptab.bytes() == 0 || rows * row_bytes >= (int64_t(1) << 32)) return false;
  return form != EBE_FORM_COLOURED || L.coff.size() > 1;
}

int product_form(const ebe_mesh* m, int order, ebe_dtype dt, int nrhs) {
  const int f = m->form[order == 2 ? 0 : 1][dt == EBE_F64 ? 0 : 1][nrhs];
  if (form_usable(m, order, f, dt, nrhs)) return f;
  return EBE_FORM_GATHER;  // untuned: the form measured fastest on the reference workloads
}

hipError_t launch_ebe_form(const ebe_mesh* m, int order, int form, ebe_dtype dt, int nrhs, const void* x, void* y,
                           bool mask_in, bool bc, bool add, const int* gate, hipStream_t s, double* gamma) {
  const PatchLevel& L = m->pl[order == 2 ? 0 : 1];
  const size_t need = size_t(L.nslots) * 3 * size_t(nrhs) * (dt == EBE_F64 ? 8 : 4);
  const int k = dt == EBE_F64 ? 0 : 1;
  const bool staged = form != EBE_FORM_COLOURED && form != EBE_FORM_ASSEMBLED;
  if ((staged && L.stage.bytes() < need) || L.npatch < 1 || nrhs < 1 || nrhs > EBE_MAX_RHS ||
      !form_usable(m, order, form, dt, nrhs) ||
      ((form == EBE_FORM_PIPELINED || form == EBE_FORM_COLOURED || form == EBE_FORM_DETERMINISTIC) &&
       !m->geo_ready[k]) ||
      (form == EBE_FORM_ASSEMBLED && !m->k1.ready[k]))
    return hipErrorInvalidValue;  // staging, geometry or assembled values not prepared, or bad form: host bug
  if (form == EBE_FORM_DETERMINISTIC)
    return launch_det(m, dt, nrhs, m->fvar[order == 2 ? 0 : 1][k][nrhs] == 1 && L.coff.size() > 1, x, y, mask_in, bc,
                      add, gate, s, gamma);
  return dt == EBE_F64 ? ebe_dispatch<double>(order, form, m, nrhs, x, y, mask_in, bc, add, gate, s, gamma)
                       : ebe_dispatch<float>(order, form, m, nrhs, x, y, mask_in, bc, add, gate, s, gamma);
}

hipError_t launch_ebe(const ebe_mesh* m, int order, ebe_dtype dt, int nrhs, const void* x, void* y, bool mask_in,
                      bool bc, bool add, const int* gate, hipStream_t s, double* gamma) {
  if (nrhs < 1 || nrhs > EBE_MAX_RHS) return hipErrorInvalidValue;
  return launch_ebe_form(m, order, product_form(m, order, dt, nrhs), dt, nrhs, x, y, mask_in, bc, add, gate, s,
                         gamma);
}

hipError_t launch_ebe_p2(const ebe_mesh* m, ebe_dtype dt, int nrhs, const void* x, void* y, bool bc,
                         hipStream_t s) {
  return launch_ebe(m, 2, dt, nrhs, x, y, bc, bc, false, nullptr, s);
}

hipError_t launch_ebe_p1(const ebe_mesh* m, ebe_dtype dt, int nrhs, const void* x, void* y, bool bc,
                         hipStream_t s) {
  return launch_ebe(m, 1, dt, nrhs, x, y, bc, bc, false, nullptr, s);
}

hipError_t launch_asm_half(const ebe_mesh* m, int level, int nrhs, const float* x, float* y, bool mask_in, bool bc,
                           bool add, const int* gate, hipStream_t s, double* gamma) {
  const AsmOp& op = level == 2 ? m->a2 : m->k1;
  if (nrhs < 1 || nrhs > EBE_MAX_RHS || (level != 1 && level != 2) || !op.ready16 || op.rows < 1)
    return hipErrorInvalidValue;  // values not prepared: host bug
  const uint8_t* fix = level == 2 ? m->cfix.as<uint8_t>() : m->fix.as<uint8_t>();
  switch (nrhs) {
#define EBE_CASE(n) \
  case n: return launch_asm_half_p<n>(m, op, fix, x, y, mask_in, bc, add, gate, s, gamma);
    EBE_CASE(1) EBE_CASE(2) EBE_CASE(3) EBE_CASE(4) EBE_CASE(5) EBE_CASE(6) EBE_CASE(7) EBE_CASE(8)
    EBE_CASE(9) EBE_CASE(10) EBE_CASE(11) EBE_CASE(12) EBE_CASE(13) EBE_CASE(14) EBE_CASE(15) EBE_CASE(16)
#undef EBE_CASE
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_level2(const ebe_mesh* m, ebe_dtype dt, int nrhs, const void* x, void* y, bool mask_in, bool bc,
                         bool add, const int* gate, hipStream_t s, double* gamma) {
  if (nrhs < 1 || nrhs > EBE_MAX_RHS || !m->a2.ready[dt == EBE_F64 ? 0 : 1] || m->n_agg < 1)
    return hipErrorInvalidValue;  // values not prepared: host bug
  const uint8_t* cf = m->cfix.as<uint8_t>();
  switch (nrhs) {
#define EBE_CASE(n)                                                                                        \
  case n:                                                                                                  \
    return dt == EBE_F64 ? launch_asm_p<double, n>(m, m->a2, cf, x, y, mask_in, bc, add, gate, s, gamma)  \
                         : launch_asm_p<float, n>(m, m->a2, cf, x, y, mask_in, bc, add, gate, s, gamma);
    EBE_CASE(1) EBE_CASE(2) EBE_CASE(3) EBE_CASE(4) EBE_CASE(5) EBE_CASE(6) EBE_CASE(7) EBE_CASE(8)
    EBE_CASE(9) EBE_CASE(10) EBE_CASE(11) EBE_CASE(12) EBE_CASE(13) EBE_CASE(14) EBE_CASE(15) EBE_CASE(16)
#undef EBE_CASE
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ebe
