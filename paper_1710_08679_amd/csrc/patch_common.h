// Helpers shared by the EBE patch kernels (ebe_kernels.hip and the
// pipelined / coloured forms in pipe_kernel.h): vector types, patch sizes
// and occupancy, the XCD-aware patch mapping, the (x, K x) fold, and the
// node-centric pass that adds staged partial sums of shared nodes.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <type_traits>

#include "ebe_internal.h"
#include "p2_element.h"

namespace ebe {
namespace {


// Size of the MI355X last-level (Infinity) cache shared by all XCDs.
constexpr int64_t kStreamStageBytes = int64_t(256) << 20;

template <typename T, int VW>
struct alignas(sizeof(T) * VW) VecT {
  T v[VW];
};

// Non-temporal (streaming) vector store and load, for the staged partial
// sums of shared nodes when a product's staging area is larger than the
// last-level cache and would only push the input vector out of the caches.
template <typename T, int VW>
__device__ __forceinline__ void store_stream(T* p, const VecT<T, VW>& v) {
  typedef T NV __attribute__((ext_vector_type(VW)));
  static_assert(sizeof(NV) == sizeof(VecT<T, VW>), "vector widths 1, 2, 4 only");
  NV r;
  __builtin_memcpy(&r, &v, sizeof(r));
  __builtin_nontemporal_store(r, reinterpret_cast<NV*>(p));
}
template <typename T, int VW>
__device__ __forceinline__ VecT<T, VW> load_stream(const T* p) {
  typedef T NV __attribute__((ext_vector_type(VW)));
  static_assert(sizeof(NV) == sizeof(VecT<T, VW>), "vector widths 1, 2, 4 only");
  const NV r = __builtin_nontemporal_load(reinterpret_cast<const NV*>(p));
  VecT<T, VW> out;
  __builtin_memcpy(&out, &r, sizeof(out));
  return out;
}

// widest vector (at most 16 bytes) whose width divides both n and the pass
// width, so every vector of a node row lies inside one pass and is aligned
constexpr int pass_vec(int nr, int cw, int value_bytes) {
  int v = 16 / value_bytes;
  while (v > 1 && (nr % v != 0 || cw % v != 0)) v /= 2;
  return v;
}

template <typename T> struct Pair;
template <> struct Pair<double> { using type = double2; };
template <> struct Pair<float> { using type = float2; };

// Cases per pass of the staged form on the quadratic mesh: at most
// EBE_P2_PASS_F32 / _F64, in passes of equal width, so that a 192-node
// patch's staged rows and FP64 accumulator fit the occupancy the form is
// built for.  The gather form and the linear mesh (<= 64 corners) take all n
// cases in one pass.
#ifndef EBE_P2_PASS_F32
#define EBE_P2_PASS_F32 8
#endif
#ifndef EBE_P2_PASS_F64
#define EBE_P2_PASS_F64 8
#endif
constexpr int chunk_for(int nr, int order, int value_bytes, bool stage) {
  const int widest = value_bytes == 8 ? EBE_P2_PASS_F64 : EBE_P2_PASS_F32;
  const int passes = (nr + widest - 1) / widest;
  return (order == 1 || !stage) ? nr : (nr + passes - 1) / passes;
}

// one work-item per (element, case) of a pass, at most kPatchThreads
// (kPatchThreadsF64 for quadratic FP64 patches)
constexpr int threads_for(int nr, int order, int value_bytes, bool stage) {
  const int want = ((order == 2 ? kPatchElems : kLinPatchElems) * chunk_for(nr, order, value_bytes, stage) + 63) /
                   64 * 64;
  const int cap = (order == 2 && value_bytes == 8) ? kPatchThreadsF64 : kPatchThreads;
  return want > cap ? cap : want;
}

// LDS of one patch workgroup and the wavefronts per SIMD that LDS leaves
// room for (160 KiB per CU, 4 SIMDs); the kernel asks the compiler for no
// more registers than that occupancy allows, but never for fewer than the
// element arithmetic needs without spilling: 128 (FP32, and the linear
// element) or 256 (quadratic FP64).  Exception: straight quadratic FP64
// patches of at most 4 cases take three wavefronts per SIMD (168 registers,
// at most 32 bytes of spills per work-item): their small workgroups are
// bound by the latency of each patch's chain of loads, not by the
// arithmetic (gather form on the 64^3 cube, one case: 0.172 -> 0.151 ms,
// two cases: 0.287 -> 0.257 ms).
template <typename T>
constexpr int patch_lds_bytes(int nr, int order, bool stage) {
  const int maxn = order == 2 ? kPatchNodes : kLinPatchCorners;
  const int wc = 3 * chunk_for(nr, order, int(sizeof(T)), stage);
  return maxn * wc * 8 + (stage ? maxn * wc * int(sizeof(T)) : 0) +
         (order == 2 ? kPatchElems : kLinPatchElems) * (14 * int(sizeof(T)) + (order == 2 ? 16 : 4)) +
         8 * maxn + 8 * nr + 16;
}
template <typename T>
constexpr int patch_waves_per_simd(int nr, int order, bool stage, bool curved = false) {
  const int lds = (patch_lds_bytes<T>(nr, order, stage) + 511) / 512 * 512;  // allocation granule
  const int wg = 163840 / lds;
  const int w = (wg > 0 ? wg : 1) * (threads_for(nr, order, int(sizeof(T)), stage) / 64) / 4;
  const int most = (sizeof(T) == 8 && order == 2) ? (nr <= 4 && !curved ? 3 : 2) : 4;
  return w > most ? most : (w < 1 ? 1 : w);
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

// Element geometry into LDS: barycentric gradients G (rows 0..3), then
// lambda s and mu s with s = V / 20 (quadratic: int L_k L_l dV = V (1 +
// delta_kl) / 20) or s = V (linear).
template <typename T, int ORDER>
__device__ __forceinline__ void store_geometry(T* __restrict__ g, const double4& p0, const double4& p1,
                                               const double4& p2, const double4& p3,
                                               const typename Pair<T>::type& lm) {
  T G[4][3];
  const T V = tet_geometry<T>(p0, p1, p2, p3, G);
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int d = 0; d < 3; ++d) g[3 * k + d] = G[k][d];
  const T s = ORDER == 2 ? V * T(0.05) : V;
  g[12] = T(lm.x) * s;
  g[13] = T(lm.y) * s;
}

// End of a patch kernel that formed (x, K x): gsum[NR] (LDS, complete) holds
// this workgroup's per-case sums.  The device-scope additions are spread over
// kGammaSlots lines (thousands of workgroups adding to one line serialise on
// it); the last workgroup to arrive folds the slots into gamma, clearing them
// as it reads.  Every access of this protocol is a device-scope atomic, so no
// fence is needed (an agent-scope fence writes back the XCD's L2, which costs
// far more than the product when every workgroup does it): a work-item waits
// for the value its addition returns, which proves the addition done, before
// the workgroup arrives at the counter.  Called by every work-item.
template <int NR, int TPB>
__device__ void fold_gamma(double* __restrict__ gsum, double* __restrict__ gamma, double* __restrict__ gslot,
                           unsigned* __restrict__ gcount) {
  __shared__ bool last;
  const int tid = threadIdx.x;
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

// values per 16-byte vector that divide a node row of 3 n values
template <typename T, int NR>
constexpr int reduce_width() {
  return (16 / int(sizeof(T)) == 4 && (3 * NR) % 4 == 0) ? 4 : ((3 * NR) % 2 == 0 ? 2 : 1);
}

template <typename T, int NR>
__global__ __launch_bounds__(256) void k_reduce_shared(const int32_t* __restrict__ snode,
                                                       const int32_t* __restrict__ soff,
                                                       const T* __restrict__ stage, int stream,
                                                       T* __restrict__ y, int32_t nshared, int bc, int add,
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
  auto ld = [&](int32_t jj) { return stream ? load_stream<T, VW>(sp + jj * W) : *reinterpret_cast<const V*>(sp + jj * W); };
  int32_t j = j0;
  for (; j + 2 <= j1; j += 2) {
    const V a = ld(j);
    const V b = ld(j + 1);
#pragma unroll
    for (int t = 0; t < VW; ++t) acc[t] += double(a.v[t]) + double(b.v[t]);
  }
  if (j < j1) {
    const V a = ld(j);
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

}  // namespace

// Pipelined (and, on the quadratic mesh, coloured) forms of the EBE product
// (pipe_kernel.h; instantiated in ebe_pipe_{f32,f64}_{lds,row}.hip).
// colour: the coloured form (order 2 only); GEO: element geometry kept in
// LDS (else read per work-item); NP: passes over the cases (instantiated: 1).
// The caller checks form_usable() first.
template <typename T, int NR, int ORDER, bool GEO, int NP>
hipError_t launch_pipe(const ebe_mesh* m, const void* x, void* y, bool mask_in, bool bc, bool add, const int* gate,
                       hipStream_t s, double* gamma, bool colour);

}  // namespace ebe
