// Deterministic form of the quadratic EBE product (Section 2, Eq. (3)): the
// same patches, element operator and shared-node staging as the gather form,
// but no atomics anywhere in the sums, so y = K x is the same bit for bit on
// every run.
//
// Per patch and pass of cases:
//   1. one work-item per (element, case) streams the element's nodal values
//      from x through K_e (p2_apply) and stores each nodal force into its own
//      slot of an element-local LDS buffer EB[element][local node][c][case]
//      (no two work-items write one slot);
//   2. after a barrier, one work-item per (patch node, component, VEC
//      consecutive cases) adds the slots of the node's incidence list (the
//      (element, local node) pairs that touch it, in element order, built on
//      the host) in FP64, in that fixed order, and writes the sums once, as
//      one vector: exclusive nodes straight into y, shared nodes into their
//      staging slot;
// and the node-centric pass adds a shared node's staged partials in patch
// order, as for the gather form.  Coloured variant: the patches run colour by
// colour (no two patches of a colour share a node), one launch per colour,
// and each patch writes its node sums straight into y, storing where it is
// the first in colour order to touch the node and adding otherwise: no
// staging and no second pass, and the additions reach a node in the fixed
// colour order.  The element buffer holds PE x 30 x CW
// values of the dtype, so the cases go in passes of CW (at most 8 in FP32,
// 4 in FP64: 48 KB).  The (x, K x) sums of the solver's products are still
// folded with device atomics (not part of y).
#include <hip/hip_runtime.h>

#include "ebe_internal.h"
#include "p2_element.h"
#include "patch_common.h"

namespace ebe {
namespace {

constexpr int kDetBufBytes = 48 * 1024;

// cases per pass: equal passes of at most kDetBufBytes of element slots
constexpr int det_cases(int nr, int vb) {
  const int wmax = kDetBufBytes / (kPatchElems * 30 * vb);
  const int passes = (nr + wmax - 1) / wmax;
  return (nr + passes - 1) / passes;
}
constexpr int det_threads(int nr, int vb) {
  const int want = (kPatchElems * det_cases(nr, vb) + 63) / 64 * 64;
  const int cap = vb == 8 ? kPatchThreadsF64 : kPatchThreads;
  return want > cap ? cap : want;
}
template <typename T>
constexpr int det_lds_bytes(int nr) {
  return kPatchElems * 30 * det_cases(nr, int(sizeof(T))) * int(sizeof(T)) + kPatchElems * 14 * int(sizeof(T)) +
         8 * kPatchNodes + 2 * (kPatchElems * 10 + kPatchNodes + 1) + 8 * nr + 64;
}
template <typename T>
constexpr int det_waves_per_simd(int nr) {
  const int lds = (det_lds_bytes<T>(nr) + 511) / 512 * 512;
  const int wg = 163840 / lds;
  const int w = (wg > 0 ? wg : 1) * (det_threads(nr, int(sizeof(T))) / 64) / 4;
  const int most = sizeof(T) == 8 ? 2 : 4;
  return w > most ? most : (w < 1 ? 1 : w);
}

// MASK, bc, add, gamma as in the gather form.  gcache: the mesh's geometry
// cache (required).  pistart: per patch entry, the start of its incidence
// list relative to the patch's first element slot; pinc: element slots
// (element - e0) * 10 + a grouped by patch entry.  COLOUR: the workgroups
// run the patches plist[0..gridDim.x) of one colour, pnode holds the
// coloured node words (bit 31: an earlier colour wrote the node).
template <typename T, int NR, bool MASK, bool COLOUR>
__global__ __launch_bounds__(det_threads(NR, int(sizeof(T))))
__attribute__((amdgpu_waves_per_eu(det_waves_per_simd<T>(NR)))) void k_ebe_det(
    const uint8_t* __restrict__ lconn, const int32_t* __restrict__ pelem, const int32_t* __restrict__ poff,
    const int32_t* __restrict__ pnode, const int32_t* __restrict__ pslot, const int32_t* __restrict__ pistart,
    const uint16_t* __restrict__ pinc, const T* __restrict__ gcache, const T* __restrict__ x, T* __restrict__ y,
    T* __restrict__ stage, int stream, int bc, int add, double* __restrict__ gamma, double* __restrict__ gslot,
    unsigned* __restrict__ gcount, const int* __restrict__ gate, const int32_t* __restrict__ plist) {
  constexpr int CW = det_cases(NR, int(sizeof(T)));
  constexpr int NPASS = (NR + CW - 1) / CW;
  constexpr int W = 3 * NR;
  constexpr int SL = 3 * CW;  // values of one (element, local node) slot row
  constexpr int VEC = pass_vec(NR, CW, int(sizeof(T)));  // cases per node-sum work-item (one vector)
  constexpr int NVR = CW / VEC;                           // vectors per component row
  using V = VecT<T, VEC>;
  constexpr int TPB = det_threads(NR, int(sizeof(T)));
  constexpr int PE = kPatchElems;
  constexpr int MAXN = kPatchNodes;
  __shared__ __align__(16) T EB[PE * 10 * SL];
  __shared__ T geo[PE][14];
  __shared__ int32_t words[MAXN];
  __shared__ int32_t slots[MAXN];
  __shared__ uint16_t inc[PE * 10];
  __shared__ uint16_t ioff[MAXN + 1];
  __shared__ double gsum[NR];
  if (gate && *gate == 0) return;
  const int tid = threadIdx.x;
  const int p = COLOUR ? plist[xcd_patch(blockIdx.x, gridDim.x)] : xcd_patch(blockIdx.x, gridDim.x);
  const int e0 = pelem[p], ne = pelem[p + 1] - e0;
  const int o0 = poff[p], nn = poff[p + 1] - o0;
  for (int i = tid; i < nn; i += TPB) {
    words[i] = pnode[o0 + i];
    slots[i] = pslot[o0 + i];
    ioff[i] = uint16_t(pistart[o0 + i]);
  }
  if (tid == 0) ioff[nn] = uint16_t(ne * 10);
  for (int k = tid; k < ne * 10; k += TPB) inc[k] = pinc[int64_t(e0) * 10 + k];
  if (tid < NR) gsum[tid] = 0.0;
  for (int el = tid; el < ne; el += TPB) {
    const T* g = gcache + (int64_t(e0) + el) * 16;
#pragma unroll
    for (int i = 0; i < 12; ++i) geo[el][i] = g[i];
    const T sv = g[12] * T(0.05);
    geo[el][12] = g[13] * sv;
    geo[el][13] = g[14] * sv;
  }
  constexpr bool kLaneCase = (64 % CW) == 0 && (TPB % CW) == 0;
  const int nj = spread_count<CW>(ne);
  __syncthreads();
#pragma unroll 1
  for (int pass = 0; pass < NPASS; ++pass) {
    const int c0 = pass * CW;
    const int cw = NR - c0 < CW ? NR - c0 : CW;
    double en_acc = 0.0;
    for (int w = tid; w < nj * CW; w += TPB) {
      const int j = w / CW;
      const int r = w - j * CW;
      const int el = spread_element<CW>(j, ne);
      if (el >= ne || r >= cw) continue;
      const int64_t e = int64_t(e0) + el;
      int gw[10];
      {
        const uint4 q = *reinterpret_cast<const uint4*>(lconn + e * 16);
        const uint32_t qw[3] = {q.x, q.y, q.z};
#pragma unroll
        for (int a = 0; a < 10; ++a) gw[a] = words[(qw[a >> 2] >> (8 * (a & 3))) & 0xff];
      }
      T G[4][3];
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int d = 0; d < 3; ++d) G[k][d] = geo[el][3 * k + d];
      const T cl = geo[el][12], cm = geo[el][13];
      T en = T(0);
      auto u = [&](int a, int c) -> T {
        const T v = x[size_t(uint32_t(gw[a]) & uint32_t(kIdxMask)) * W + c * NR + c0 + r];
        return (MASK && ((gw[a] >> (kIdxBits + c)) & 1)) ? T(0) : v;
      };
      T* eb = EB + (el * 10) * SL + r;
      auto emit = [&](int a, const T f[3]) {
#pragma unroll
        for (int c = 0; c < 3; ++c) eb[a * SL + c * CW] = f[c];
      };
      p2_apply<T>(G, cl, cm, u, emit, gamma != nullptr, en);
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
    // node sums in incidence order; items (entry, component, vector of
    // cases), cases fastest.  Vectors never straddle the pass's last case
    // (VEC divides both n and the pass width).
    for (int w = tid; w < nn * 3 * NVR; w += TPB) {
      const int ent = w / (3 * NVR);
      const int rem = w - ent * (3 * NVR);
      const int c = rem / NVR, r0 = (rem - c * NVR) * VEC;
      if (r0 >= cw) continue;
      double s[VEC];
#pragma unroll
      for (int t = 0; t < VEC; ++t) s[t] = 0.0;
      const int k1 = ioff[ent + 1];
      for (int k = ioff[ent]; k < k1; ++k) {
        const V v = *reinterpret_cast<const V*>(EB + int(inc[k]) * SL + c * CW + r0);
#pragma unroll
        for (int t = 0; t < VEC; ++t) s[t] += double(v.v[t]);
      }
      V out;
#pragma unroll
      for (int t = 0; t < VEC; ++t) out.v[t] = T(s[t]);
      const int32_t wd = words[ent];
      const int col = c * NR + c0 + r0;
      if (!COLOUR && wd < 0) {  // shared node: partial sums to its staging slot
        T* sp = stage + size_t(slots[ent]) * W + col;
        if (stream) store_stream<T, VEC>(sp, out);
        else *reinterpret_cast<V*>(sp) = out;
      } else {
        V* yp = reinterpret_cast<V*>(y + size_t(wd & kIdxMask) * W + col);
        const bool fixed = bc && ((wd >> (kIdxBits + c)) & 1);
        if (add || (COLOUR && wd < 0)) {  // y += (the caller, or an earlier colour, wrote y)
          if (!fixed) {  // (a fixed DOF keeps the caller's value or the first colour's zero)
            V o = *yp;
#pragma unroll
            for (int t = 0; t < VEC; ++t) o.v[t] += out.v[t];
            *yp = o;
          }
        } else {
          if (fixed) {
#pragma unroll
            for (int t = 0; t < VEC; ++t) out.v[t] = T(0);
          }
          *yp = out;
        }
      }
    }
    if (pass + 1 < NPASS) __syncthreads();  // EB is refilled by the next pass
  }
  if (gamma) fold_gamma<NR, TPB>(gsum, gamma, gslot, gcount);
}

template <typename T, int NR, bool MASK, bool COLOUR>
hipError_t launch_det_k(const ebe_mesh* m, const int32_t* plist, int64_t npatch, const void* x, void* y, bool st,
                        bool bc, bool add, const int* gate, hipStream_t s, double* gamma) {
  const PatchLevel& L = m->pl[0];
  const int k = sizeof(T) == 8 ? 0 : 1;
  unsigned* gcount = reinterpret_cast<unsigned*>(m->gacc.as<char>() + kGammaBytes - 64);
  hipLaunchKernelGGL((k_ebe_det<T, NR, MASK, COLOUR>), dim3(unsigned(npatch)), dim3(det_threads(NR, int(sizeof(T)))),
                     0, s, m->lconn.as<uint8_t>(), L.pelem.as<int32_t>(), L.poff.as<int32_t>(),
                     COLOUR ? L.cword.as<int32_t>() : L.pnode.as<int32_t>(), L.pslot.as<int32_t>(),
                     L.pistart.as<int32_t>(), L.pinc.as<uint16_t>(), m->geo[k].as<T>(), static_cast<const T*>(x),
                     static_cast<T*>(y), L.stage.as<T>(), int(st), int(bc), int(add), gamma, m->gacc.as<double>(),
                     gcount, gate, plist);
  return hipGetLastError();
}

template <typename T, int NR, bool COLOUR>
hipError_t launch_det_m(const ebe_mesh* m, const int32_t* plist, int64_t npatch, const void* x, void* y, bool st,
                        bool mask_in, bool bc, bool add, const int* gate, hipStream_t s, double* gamma) {
  return mask_in ? launch_det_k<T, NR, true, COLOUR>(m, plist, npatch, x, y, st, bc, add, gate, s, gamma)
                 : launch_det_k<T, NR, false, COLOUR>(m, plist, npatch, x, y, st, bc, add, gate, s, gamma);
}

template <typename T, int NR>
hipError_t launch_det_p(const ebe_mesh* m, bool colour, const void* x, void* y, bool mask_in, bool bc, bool add,
                        const int* gate, hipStream_t s, double* gamma) {
  const PatchLevel& L = m->pl[0];
  if (colour) {  // colours in turn, sums straight into y
    const int32_t* cp = L.cperm.as<int32_t>();
    for (size_t c = 0; c + 1 < L.coff.size(); ++c) {
      const hipError_t e = launch_det_m<T, NR, true>(m, cp + L.coff[c], L.coff[c + 1] - L.coff[c], x, y, false,
                                                     mask_in, bc, add, gate, s, gamma);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  const bool st = int64_t(L.nslots) * 3 * NR * int64_t(sizeof(T)) > kStreamStageBytes;
  hipError_t e = launch_det_m<T, NR, false>(m, nullptr, L.npatch, x, y, st, mask_in, bc, add, gate, s, gamma);
  if (e != hipSuccess || L.nshared == 0) return e;
  const int64_t work = L.nshared * (3 * NR / reduce_width<T, NR>());
  hipLaunchKernelGGL((k_reduce_shared<T, NR>), dim3(unsigned((work + 255) / 256)), dim3(256), 0, s,
                     L.snode.as<int32_t>(), L.soff.as<int32_t>(), L.stage.as<T>(), int(st), static_cast<T*>(y),
                     int32_t(L.nshared), int(bc), int(add), gate);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_det(const ebe_mesh* m, ebe_dtype dt, int nrhs, bool colour, const void* x, void* y, bool mask_in,
                      bool bc, bool add, const int* gate, hipStream_t s, double* gamma) {
  if (m->pl[0].npatch < 1 || m->pl[0].pinc.bytes() == 0 || !m->geo_ready[dt == EBE_F64 ? 0 : 1] ||
      (colour && m->pl[0].coff.size() < 2))
    return hipErrorInvalidValue;  // tables or geometry not prepared: host bug
  switch (nrhs) {
#define EBE_CASE(n)                                                                                       \
  case n:                                                                                                 \
    return dt == EBE_F64 ? launch_det_p<double, n>(m, colour, x, y, mask_in, bc, add, gate, s, gamma)    \
                         : launch_det_p<float, n>(m, colour, x, y, mask_in, bc, add, gate, s, gamma);
    EBE_CASE(1) EBE_CASE(2) EBE_CASE(3) EBE_CASE(4) EBE_CASE(5) EBE_CASE(6) EBE_CASE(7) EBE_CASE(8)
    EBE_CASE(9) EBE_CASE(10) EBE_CASE(11) EBE_CASE(12) EBE_CASE(13) EBE_CASE(14) EBE_CASE(15) EBE_CASE(16)
#undef EBE_CASE
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ebe
