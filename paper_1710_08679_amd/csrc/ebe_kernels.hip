// Element-by-element products on gfx950 (Section 2, Eq. (3)): y = K x for the
// quadratic mesh and y = K1 x for the linear (corner) mesh, n cases at once.
//
// Work decomposition (see patches.cpp).  One workgroup per element patch
// (<= 64 elements, <= 192 nodes):
//   1. the patch's node words (id, Dirichlet bits, shared flag) and staging
//      slots go to LDS, together with a cleared FP64 force accumulator
//      F[node][component][case];
//   2. one work-item per element rebuilds the element geometry from the four
//      corner coordinates and material (the element matrix is never stored,
//      Section 2) and keeps it in LDS;
//   3. one work-item per (element, case) gathers its nodal values (the n
//      cases of a node are contiguous: Section 3.1's coalesced case loop),
//      forms K_e u_e in registers (p2_element.h) and adds the forces into F
//      with LDS FP64 atomics (FP32 LDS atomics are much slower on this part);
//   4. each patch node is written once: exclusive nodes straight into y,
//      shared nodes as a partial sum into their staging slot.
// A second, node-centric kernel adds the consecutive staged partials of each
// shared node in patch order.  Global memory sees no atomics, every node is
// written exactly once per product (so y needs no clearing pass), and the
// result does not depend on scheduling.
#include <hip/hip_runtime.h>

#include "ebe_internal.h"
#include "p2_element.h"

namespace ebe {
namespace {

template <typename T> struct Pair;
template <> struct Pair<double> { using type = double2; };
template <> struct Pair<float> { using type = float2; };

constexpr int threads_for(int nr) {
  return (kPatchElems * nr + 63) / 64 * 64 > kPatchThreads ? kPatchThreads : (kPatchElems * nr + 63) / 64 * 64;
}

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own
// L2.  Give XCD x the contiguous patch range [start_x, start_x + count_x), so
// that neighbouring patches, which share about half their nodes, read those
// nodes through the same L2.  A bijection on [0, npatch).
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_patch(int b, int npatch) {
  const int x = b % kXcds, i = b / kXcds;
  const int q = npatch / kXcds, rr = npatch % kXcds;
  return x * q + (x < rr ? x : rr) + i;
}

// Within a wave the cases of an element occupy adjacent lanes, so a wave
// holds 64 / n elements.  Consecutive elements of a patch (tetrahedra of one
// hexahedron in a structured mesh) share many nodes, and their LDS atomics
// then hit the same address in one instruction.  Interleaving by a stride of
// ceil(ne / G) spreads a wave's elements over the patch.
// Items j in [0, spread_count) map to elements spread_element(j) (>= ne: skip).
template <int NR>
__device__ __forceinline__ int spread_count(int ne) {
  constexpr int G = 64 / NR;  // elements per wave
  return G <= 1 ? ne : ((ne + G - 1) / G) * G;
}
template <int NR>
__device__ __forceinline__ int spread_element(int j, int ne) {
  constexpr int G = 64 / NR;
  if constexpr (G <= 1) {
    return j;
  } else {
    const int K = (ne + G - 1) / G;
    return (j % G) * K + j / G;
  }
}

// MASK_IN: zero the fixed DOFs of x while gathering (y = P K P x); callers
// whose x is already zero there (the solver) skip it.  bc: zero the fixed
// DOFs of y.  add: y += K x instead of y = K x.  gamma (optional): gamma[r]
// += (x_r, K x_r) formed element by element as sum_e x_eᵀ K_e x_e, which is
// what CG needs from q = K p without a separate inner-product pass.
template <typename T, int NR, int ORDER, bool MASK_IN>
__global__ __launch_bounds__(threads_for(NR)) void k_ebe_patch(
    const int32_t* __restrict__ conn, const uint8_t* __restrict__ lconn, const int32_t* __restrict__ pelem,
    const int32_t* __restrict__ poff, const int32_t* __restrict__ pnode, const int32_t* __restrict__ pslot,
    const double4* __restrict__ xv, const typename Pair<T>::type* __restrict__ lame, const T* __restrict__ x,
    T* __restrict__ y, T* __restrict__ stage, int bc, int add, double* __restrict__ gamma,
    double* __restrict__ gslot, unsigned* __restrict__ gcount, const int* __restrict__ gate) {
  constexpr int NLOC = ORDER == 2 ? 10 : 4;
  constexpr int W = 3 * NR;
  constexpr int TPB = threads_for(NR);
  constexpr int MAXN = ORDER == 2 ? kPatchNodes : kPatchCorners;
  constexpr int EPP = TPB / W;  // patch nodes written per pass
  __shared__ double F[MAXN * W];
  __shared__ T geo[kPatchElems][14];
  __shared__ int32_t words[MAXN];
  __shared__ int32_t slots[MAXN];
  __shared__ double gsum[NR];
  if (gate && *gate == 0) return;
  const int tid = threadIdx.x;
  const int p = xcd_patch(blockIdx.x, gridDim.x);
  const int e0 = pelem[p], ne = pelem[p + 1] - e0;
  const int o0 = poff[p], nn = poff[p + 1] - o0;
  for (int i = tid; i < nn * W; i += TPB) F[i] = 0.0;
  if (tid < NR) gsum[tid] = 0.0;
  for (int i = tid; i < nn; i += TPB) {
    words[i] = pnode[o0 + i];
    slots[i] = pslot[o0 + i];
  }
  for (int el = tid; el < ne; el += TPB) {
    const int64_t e = int64_t(e0) + el;
    T G[4][3];
    const T V = tet_geometry<T>(xv[conn[e * 10 + 0] & kIdxMask], xv[conn[e * 10 + 1] & kIdxMask],
                                xv[conn[e * 10 + 2] & kIdxMask], xv[conn[e * 10 + 3] & kIdxMask], G);
    const auto lm = lame[e];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int d = 0; d < 3; ++d) geo[el][3 * k + d] = G[k][d];
    const T s = ORDER == 2 ? V * T(0.05) : V;  // int L_k L_l dV = V (1 + delta_kl) / 20
    geo[el][12] = T(lm.x) * s;
    geo[el][13] = T(lm.y) * s;
  }
  __syncthreads();
  // (x, K x) contributions: when n divides 64 a work-item keeps one case for
  // all its items, so it sums them in a register and the lanes of a case are
  // combined across the wavefront before one LDS atomic per case.
  constexpr bool kLaneCase = (64 % NR) == 0;
  double en_acc = 0.0;
  const int nj = spread_count<NR>(ne);
  for (int w = tid; w < nj * NR; w += TPB) {
    const int j = w / NR;
    const int r = w - j * NR;
    const int el = spread_element<NR>(j, ne);
    if (el >= ne) continue;
    const int64_t e = int64_t(e0) + el;
    int lid[NLOC];
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
    T G[4][3];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int d = 0; d < 3; ++d) G[k][d] = geo[el][3 * k + d];
    const T cl = geo[el][12], cm = geo[el][13];
    T u[NLOC][3];
#pragma unroll
    for (int a = 0; a < NLOC; ++a) {
      const int32_t wd = words[lid[a]];
      const T* xp = x + size_t(uint32_t(wd) & uint32_t(kIdxMask)) * W + r;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        T v = xp[c * NR];
        if constexpr (MASK_IN) v = ((wd >> (kIdxBits + c)) & 1) ? T(0) : v;
        u[a][c] = v;
      }
    }
    T f[NLOC][3];
    if constexpr (ORDER == 2)
      p2_forces<T>(G, cl, cm, reinterpret_cast<const T(*)[3]>(u), reinterpret_cast<T(*)[3]>(f));
    else
      p1_forces<T>(G, cl, cm, reinterpret_cast<const T(*)[3]>(u), reinterpret_cast<T(*)[3]>(f));
#pragma unroll
    for (int a = 0; a < NLOC; ++a) {
      double* fp = F + lid[a] * W + r;
#pragma unroll
      for (int c = 0; c < 3; ++c) atomicAdd(fp + c * NR, double(f[a][c]));
    }
    if (gamma) {
      T en = T(0);
#pragma unroll
      for (int a = 0; a < NLOC; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c) en += u[a][c] * f[a][c];
      if constexpr (kLaneCase) en_acc += double(en);
      else atomicAdd(&gsum[r], double(en));
    }
  }
  if constexpr (kLaneCase) {
    if (gamma) {
#pragma unroll
      for (int off = 32; off >= NR; off >>= 1) en_acc += __shfl_xor(en_acc, off, 64);
      if ((tid & 63) < NR) atomicAdd(&gsum[tid & 63], en_acc);
    }
  }
  __syncthreads();
  const int eo = tid / W;
  const int rem = tid - eo * W;
  const int c = rem / NR;
  if (eo < EPP) {
    for (int ent = eo; ent < nn; ent += EPP) {
      const int32_t wd = words[ent];
      const T v = T(F[ent * W + rem]);
      if (wd < 0) {  // shared node: partial sum to its staging slot
        stage[size_t(slots[ent]) * W + rem] = v;
      } else {
        T* yp = y + size_t(wd & kIdxMask) * W + rem;
        const bool fixed = bc && ((wd >> (kIdxBits + c)) & 1);
        if (add) {
          if (!fixed) *yp += v;
        } else {
          *yp = fixed ? T(0) : v;
        }
      }
    }
  }
  if (!gamma) return;
  // Spread the device-scope additions over kGammaSlots lines (thousands of
  // workgroups adding to one line serialise on it), then let the last
  // workgroup to arrive fold the slots into gamma, clearing them as it reads.
  // Every access of this protocol is a device-scope atomic, so no fence is
  // needed (an agent-scope fence writes back the XCD's L2, which costs far
  // more than the product when every workgroup does it): a work-item waits
  // for the value its addition returns, which proves the addition done,
  // before the workgroup arrives at the counter.
  __shared__ bool last;
  if (tid < NR) {
    const double old = __hip_atomic_fetch_add(gslot + (blockIdx.x % kGammaSlots) * EBE_MAX_RHS + tid, gsum[tid],
                                              __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    asm volatile("" ::"v"(old));
  }
  __syncthreads();
  if (tid == 0) last = atomicAdd(gcount, 1u) == gridDim.x - 1;
  __syncthreads();
  if (!last) return;
  if (tid < NR) gsum[tid] = 0.0;
  __syncthreads();
  for (int i = tid; i < kGammaSlots * NR; i += TPB) {
    const int sl = i / NR, r = i - sl * NR;
    atomicAdd(&gsum[r], atomicExch(gslot + sl * EBE_MAX_RHS + r, 0.0));
  }
  __syncthreads();
  if (tid < NR) unsafeAtomicAdd(gamma + tid, gsum[tid]);
  if (tid == 0) atomicExch(gcount, 0u);
}

// y[shared node] (=|+=) sum of its consecutive staged partials (patch order).
// The host guarantees nshared * 3 * NR < 2^31 and nslots * 3 * NR < 2^31.
template <typename T, int VW>
struct alignas(sizeof(T) * VW) VecT {
  T v[VW];
};

// values per 16-byte vector that divide a node row of 3 n values
template <typename T, int NR>
constexpr int reduce_width() {
  return (16 / int(sizeof(T)) == 4 && (3 * NR) % 4 == 0) ? 4 : ((3 * NR) % 2 == 0 ? 2 : 1);
}

template <typename T, int NR>
__global__ __launch_bounds__(256) void k_reduce_shared(const int32_t* __restrict__ snode,
                                                       const int32_t* __restrict__ soff,
                                                       const T* __restrict__ stage, T* __restrict__ y,
                                                       int32_t nshared, int bc, int add,
                                                       const int* __restrict__ gate) {
  constexpr int W = 3 * NR;
  constexpr int VW = reduce_width<T, NR>();
  constexpr int U = W / VW;  // work-items per shared node
  using V = VecT<T, VW>;
  if (gate && *gate == 0) return;
  const int32_t i = int32_t(blockIdx.x) * 256 + int32_t(threadIdx.x);
  if (i >= nshared * U) return;
  const int32_t k = i / U;
  const int32_t rem = (i - k * U) * VW;
  const int32_t wd = snode[k];
  const int32_t j0 = soff[k], j1 = soff[k + 1];
  const T* sp = stage + rem;
  double acc[VW];
#pragma unroll
  for (int t = 0; t < VW; ++t) acc[t] = 0.0;
  int32_t j = j0;
  for (; j + 2 <= j1; j += 2) {
    const V a = *reinterpret_cast<const V*>(sp + j * W);
    const V b = *reinterpret_cast<const V*>(sp + (j + 1) * W);
#pragma unroll
    for (int t = 0; t < VW; ++t) acc[t] += double(a.v[t]) + double(b.v[t]);
  }
  if (j < j1) {
    const V a = *reinterpret_cast<const V*>(sp + j * W);
#pragma unroll
    for (int t = 0; t < VW; ++t) acc[t] += double(a.v[t]);
  }
  V* yp = reinterpret_cast<V*>(y + size_t(wd & kIdxMask) * W + rem);
  V out = add ? *yp : V{};
#pragma unroll
  for (int t = 0; t < VW; ++t) {
    const int c = (rem + t) / NR;
    const bool fixed = bc && ((wd >> (kIdxBits + c)) & 1);
    if (add) {
      if (!fixed) out.v[t] += T(acc[t]);
    } else {
      out.v[t] = fixed ? T(0) : T(acc[t]);
    }
  }
  *yp = out;
}

template <typename T, int NR, int ORDER, bool MASK_IN>
void launch_patch(const ebe_mesh* m, const PatchLevel& L, const void* x, void* y, T* stage, bool bc, bool add,
                  const int* gate, hipStream_t s, double* gamma) {
  using P = typename Pair<T>::type;
  const P* lame = (sizeof(T) == 8) ? reinterpret_cast<const P*>(m->lame64.as<void>())
                                   : reinterpret_cast<const P*>(m->lame32.as<void>());
  hipLaunchKernelGGL((k_ebe_patch<T, NR, ORDER, MASK_IN>), dim3(unsigned(m->n_patch)), dim3(threads_for(NR)), 0,
                     s, m->conn.as<int32_t>(), ORDER == 2 ? m->lconn.as<uint8_t>() : m->lconn1.as<uint8_t>(),
                     m->pelem.as<int32_t>(), L.poff.as<int32_t>(), L.pnode.as<int32_t>(), L.pslot.as<int32_t>(),
                     m->xv.as<double4>(), lame, static_cast<const T*>(x), static_cast<T*>(y), stage, int(bc),
                     int(add), gamma, m->gacc.as<double>(),
                     reinterpret_cast<unsigned*>(m->gacc.as<char>() + kGammaBytes - 64), gate);
}

template <typename T, int NR>
hipError_t ebe_dispatch_p(int order, const ebe_mesh* m, const void* x, void* y, bool mask_in, bool bc, bool add,
                          const int* gate, hipStream_t s, double* gamma) {
  const PatchLevel& L = m->pl[order == 2 ? 0 : 1];
  T* stage = L.stage.as<T>();
  if (order == 2) {
    if (mask_in) launch_patch<T, NR, 2, true>(m, L, x, y, stage, bc, add, gate, s, gamma);
    else launch_patch<T, NR, 2, false>(m, L, x, y, stage, bc, add, gate, s, gamma);
  } else {
    if (mask_in) launch_patch<T, NR, 1, true>(m, L, x, y, stage, bc, add, gate, s, gamma);
    else launch_patch<T, NR, 1, false>(m, L, x, y, stage, bc, add, gate, s, gamma);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || L.nshared == 0) return e;
  const int64_t work = L.nshared * (3 * NR / reduce_width<T, NR>());
  hipLaunchKernelGGL((k_reduce_shared<T, NR>), dim3(unsigned((work + 255) / 256)), dim3(256), 0, s,
                     L.snode.as<int32_t>(), L.soff.as<int32_t>(), stage, static_cast<T*>(y), int32_t(L.nshared),
                     int(bc), int(add), gate);
  return hipGetLastError();
}

template <typename T>
hipError_t ebe_dispatch(int order, const ebe_mesh* m, int nrhs, const void* x, void* y, bool mask_in, bool bc,
                        bool add, const int* gate, hipStream_t s, double* gamma) {
  switch (nrhs) {
#define EBE_CASE(n) \
  case n: return ebe_dispatch_p<T, n>(order, m, x, y, mask_in, bc, add, gate, s, gamma);
    EBE_CASE(1) EBE_CASE(2) EBE_CASE(3) EBE_CASE(4) EBE_CASE(5) EBE_CASE(6) EBE_CASE(7) EBE_CASE(8)
    EBE_CASE(9) EBE_CASE(10) EBE_CASE(11) EBE_CASE(12) EBE_CASE(13) EBE_CASE(14) EBE_CASE(15) EBE_CASE(16)
#undef EBE_CASE
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

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

hipError_t launch_ebe(const ebe_mesh* m, int order, ebe_dtype dt, int nrhs, const void* x, void* y, bool mask_in,
                      bool bc, bool add, const int* gate, hipStream_t s, double* gamma) {
  const PatchLevel& L = m->pl[order == 2 ? 0 : 1];
  const size_t need = size_t(L.nslots) * 3 * size_t(nrhs) * (dt == EBE_F64 ? 8 : 4);
  if (L.stage.bytes() < need || m->n_patch < 1) return hipErrorInvalidValue;  // staging not sized: host bug
  return dt == EBE_F64 ? ebe_dispatch<double>(order, m, nrhs, x, y, mask_in, bc, add, gate, s, gamma)
                       : ebe_dispatch<float>(order, m, nrhs, x, y, mask_in, bc, add, gate, s, gamma);
}

hipError_t launch_ebe_p2(const ebe_mesh* m, ebe_dtype dt, int nrhs, const void* x, void* y, bool bc,
                         hipStream_t s) {
  return launch_ebe(m, 2, dt, nrhs, x, y, bc, bc, false, nullptr, s);
}

hipError_t launch_ebe_p1(const ebe_mesh* m, ebe_dtype dt, int nrhs, const void* x, void* y, bool bc,
                         hipStream_t s) {
  return launch_ebe(m, 1, dt, nrhs, x, y, bc, bc, false, nullptr, s);
}

}  // namespace ebe
