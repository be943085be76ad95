// Pipelined and coloured forms of the EBE product (Section 2, Eq. (3)).
//
// Pipelined form: a persistent workgroup works through a sequence of patches
// (those of its XCD's contiguous range, in steps of the number of workgroups
// on that XCD) and keeps the next patch's metadata in flight while it
// computes the current one.  Per patch:
//   A. commit the prefetched node words (and staging slots) to LDS, form each
//      element's node table (below) from its prefetched node words, clear
//      the FP64 accumulator F;
//   B. issue the next patch's bounds, node words and slots (and, in the
//      variant that reads the geometry per work-item, its element node
//      words);
//   C. element phase: one work-item per (element, case) reads the element's
//      geometry row (gradients, volume, lambda, mu: the mesh's geometry
//      cache, formed from the corner coordinates) and its ten nodal values,
//      streams them through K_e (p2_element.h) and adds each nodal force
//      into F with an FP64 LDS atomic;
//   D. (other variant) issue the next patch's element node words;
//   E. write back: exclusive nodes straight into y, shared nodes as partial
//      sums into their staging slots (a node-centric pass adds them after).
//
// Node table.  For each element of the patch, formed once when the patch is
// committed (one work-item per element): for each node, the byte offset of
// its row in x and y (node id x 3 n x sizeof(T)) and of its row in F (local
// id x 3 n x 8).  A work-item of the element phase then adds only its case
// offset to each: no index unpacking or multiplication per (element, case).
// The mesh's element node words (ptab: node id | local id << 25) carry
// both ids, so the table needs no lookup of the patch's node list.
//
// Coloured form (quadratic level): the patches are coloured so that no two
// patches of a colour share a node, and the colours run one launch after
// another.  A patch writes every one of its nodes straight into y: the first
// patch (in colour order) to touch a node stores its sum, the later ones add
// theirs to what y holds (node word bit 31 set).  No staging buffer, no
// second pass and no atomics in global memory, at the price of one launch
// per colour and a read of y for the nodes shared between colours.  The
// patches' sums reach a node in colour order; inside a patch they are LDS
// atomics as in the other forms (so not bitwise reproducible).
#pragma once

#include "patch_common.h"

namespace ebe {
namespace {

// Cases per pass and work-items per workgroup.  NP = 1 (the instantiated
// kernels): all n cases in one pass, the workgroup size of the other forms.
// NP = 2: the cases in two passes of n / 2, so the FP64 accumulator holds
// half the cases (32 KB per workgroup at n = 16: five workgroups per CU
// instead of two), in workgroups of two element rounds per pass (48
// elements x 8 cases on 192 work-items, no wavefront idle at the barrier
// that ends the element phase); measured slower on the 64^3 cube (FP32
// n = 16: 0.92 ms coloured, 1.16 ms pipelined, against 0.69 and 0.78 in one
// pass), so not instantiated.
template <typename T>
constexpr int pipe_threads(int nr, int order, int np) {
  if (np == 2) {
    const int items = (order == 2 ? kPatchElems : kLinPatchElems) * (nr / 2);
    return (items / 2 + 63) / 64 * 64;
  }
  return threads_for(nr, order, int(sizeof(T)), false);
}

template <typename T>
constexpr int pipe_lds_bytes(int nr, int order, bool geo_lds, int np) {
  const int maxn = order == 2 ? kPatchNodes : kLinPatchCorners;
  const int pe = order == 2 ? kPatchElems : kLinPatchElems;
  const int nloc = order == 2 ? 10 : 4;
  return maxn * 3 * (nr / np) * 8 + pe * 2 * nloc * 4 + (geo_lds ? pe * 14 * int(sizeof(T)) : 0) + 8 * maxn +
         8 * nr + 16;
}

template <typename T>
constexpr int pipe_waves_per_simd(int nr, int order, bool geo_lds, int np) {
  const int lds = (pipe_lds_bytes<T>(nr, order, geo_lds, np) + 511) / 512 * 512;
  const int wg = 163840 / lds;
  // waves per SIMD when the resident workgroups' wavefronts spread over the 4 SIMDs
  const int w = ((wg > 0 ? wg : 1) * (pipe_threads<T>(nr, order, np) / 64) + 3) / 4;
  const int most = (sizeof(T) == 8 && order == 2) ? 2 : 4;
  return w > most ? most : (w < 1 ? 1 : w);
}

// GAMMA: also form gamma[r] += (x_r, K x_r) element by element (what CG needs
// from q = K p).  MASK: zero the fixed DOFs of x while reading it.  COLOUR:
// the coloured form; plist then lists this launch's patches (one colour).
// GEO: element geometry prefetched with the patch metadata and kept in LDS
// (else each work-item of the element phase reads its element's row).  NP:
// passes over the cases (above).  Which variant is faster depends on the
// dtype and n, so the tuner measures them.
template <typename T, int NR, int ORDER, bool MASK, bool GAMMA, bool COLOUR, bool GEO, int NP>
__global__ __launch_bounds__(pipe_threads<T>(NR, ORDER, NP))
__attribute__((amdgpu_waves_per_eu(pipe_waves_per_simd<T>(NR, ORDER, GEO, NP)))) void k_ebe_pipe(
    const T* __restrict__ gcache, const uint32_t* __restrict__ ptab, const int32_t* __restrict__ pelem,
    const int32_t* __restrict__ poff, const int32_t* __restrict__ pnode, const int32_t* __restrict__ pslot,
    const int32_t* __restrict__ plist, const T* __restrict__ x, T* __restrict__ y, T* __restrict__ stage,
    int stream, int npatch, int bc, int add, double* __restrict__ gamma, double* __restrict__ gslot,
    unsigned* __restrict__ gcount, const int* __restrict__ gate) {
  static_assert(NP == 1 || NR % NP == 0, "passes split the cases evenly");
  constexpr int NLOC = ORDER == 2 ? 10 : 4;
  constexpr int W = 3 * NR;                         // values of a node row in x, y and the staging buffer
  constexpr int CW = NR / NP;                       // cases per pass
  constexpr int WC = 3 * CW;                        // values of a node row of F (one pass)
  constexpr uint32_t RB = uint32_t(W * sizeof(T));  // bytes of a node row in x and y
  constexpr uint32_t FB = uint32_t(WC * 8);         // bytes of a node row in F
  constexpr int TPB = pipe_threads<T>(NR, ORDER, NP);
  constexpr int MAXN = ORDER == 2 ? kPatchNodes : kLinPatchCorners;
  constexpr int PE = ORDER == 2 ? kPatchElems : kLinPatchElems;
  constexpr int KW = (MAXN + TPB - 1) / TPB;           // node entries per work-item
  constexpr int KE = (PE + TPB - 1) / TPB;             // elements per work-item (node tables)
  constexpr int GW = 64 / CW > 1 ? 64 / CW : 1;        // elements per wave in the element phase
  constexpr int KI = ((PE + GW - 1) / GW * GW * CW + TPB - 1) / TPB;  // element-phase items per work-item
  constexpr int VEC = pass_vec(NR, CW, int(sizeof(T)));
  constexpr int NV = WC / VEC;                          // vectors of a node row in one pass
  constexpr int EPK = TPB / NV;
  constexpr int KIT = (MAXN + EPK - 1) / EPK;
  constexpr int GV = 16 / int(sizeof(T));  // values per 16-byte piece of a geometry row
  using V = VecT<T, VEC>;
  using GR = VecT<T, GV>;
  __shared__ double F[MAXN * WC];
  __shared__ uint32_t etab[PE][2 * NLOC];  // per element: NLOC x-row byte offsets, then NLOC F-row byte offsets
  constexpr bool kGeoLds = GEO;
  __shared__ T geo[kGeoLds ? PE : 1][14];   // per element: G (12), lambda V s, mu V s
  __shared__ int32_t words[MAXN];
  __shared__ int32_t slots[COLOUR ? 1 : MAXN];
  __shared__ double gsum[NR];
  if (gate && *gate == 0) return;
  const int tid = threadIdx.x;
  // this workgroup's patches: XCD x owns [start, stop); its g-th workgroup
  // takes start + g, start + g + wx, ...
  const int G = gridDim.x, xcd = blockIdx.x % kXcds;
  const int wx = (G - xcd + kXcds - 1) / kXcds;  // workgroups on this XCD
  const int q = npatch / kXcds, rr = npatch % kXcds;
  const int start = xcd * q + (xcd < rr ? xcd : rr), stop = start + q + (xcd < rr ? 1 : 0);
  int p = start + int(blockIdx.x) / kXcds;
  if (GAMMA && tid < NR) gsum[tid] = 0.0;
  // F starts at zero; every write-back zeroes what it read, so it stays zero between passes
  for (int i = tid; i < MAXN * WC; i += TPB) F[i] = 0.0;
  // this work-item's vector of a pass's node row (write-back): value sq of the
  // row, component sc, cases scc .. scc + VEC - 1 of the pass
  const int sv = tid % NV, sent = tid < EPK * NV ? tid / NV : MAXN, sq = sv * VEC, sc = sq / CW, scc = sq - sc * CW;

  // prefetched state of the next patch
  int e0 = 0, ne = 0, o0 = 0, nn = 0;
  int pw[KW], ps[KW];
  uint32_t pt[KE][NLOC];
  GR pg[kGeoLds ? KE : 1][16 / GV];
  auto patch_id = [&](int i) { return COLOUR ? plist[i] : i; };
  auto fetch_meta = [&](int pp) {  // bounds, node words and slots of patch pp
    const int id = patch_id(pp);
    e0 = pelem[id];
    ne = pelem[id + 1] - e0;
    o0 = poff[id];
    nn = poff[id + 1] - o0;
#pragma unroll
    for (int k = 0; k < KW; ++k) {
      const int i = tid + k * TPB;
      pw[k] = i < nn ? pnode[o0 + i] : 0;
      if constexpr (!COLOUR) ps[k] = i < nn ? pslot[o0 + i] : 0;
    }
    if constexpr (kGeoLds) {
#pragma unroll
      for (int k = 0; k < KE; ++k) {
        const int el = tid + k * TPB;
        if (el < ne) {
          const GR* row = reinterpret_cast<const GR*>(gcache + (int64_t(e0) + el) * 16);
#pragma unroll
          for (int v = 0; v < 16 / GV; ++v) pg[k][v] = row[v];
        }
      }
    }
  };
  auto fetch_late = [&]() {  // node words of this work-item's elements of the prefetched patch
#pragma unroll
    for (int k = 0; k < KE; ++k) {
      const int el = tid + k * TPB;
      if (el < ne) {
        const uint32_t* row = ptab + (int64_t(e0) + el) * NLOC;
        if constexpr (NLOC == 10) {
#pragma unroll
          for (int a = 0; a < 10; a += 2) {
            const uint2 v = *reinterpret_cast<const uint2*>(row + a);
            pt[k][a] = v.x;
            pt[k][a + 1] = v.y;
          }
        } else {
          const uint4 v = *reinterpret_cast<const uint4*>(row);
          pt[k][0] = v.x;
          pt[k][1] = v.y;
          pt[k][2] = v.z;
          pt[k][3] = v.w;
        }
      }
    }
  };
  if (p < stop) {
    fetch_meta(p);
    fetch_late();
  }
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): the first commit, as every later one, finds its loads done
  // (x, K x): a work-item keeps one case of each pass when the pass width
  // divides 64, so it sums in registers (one sum per pass) and the lanes of a
  // case are combined across the wavefront at the end
  constexpr bool kLaneCase = (64 % CW) == 0 && (TPB % CW) == 0;
  double en_acc[NP];
#pragma unroll
  for (int ps_ = 0; ps_ < NP; ++ps_) en_acc[ps_] = 0.0;
#pragma unroll 1
  for (; p < stop; p += wx) {
    // A. commit this patch
#pragma unroll
    for (int k = 0; k < KW; ++k) {
      const int i = tid + k * TPB;
      if (i < nn) {
        words[i] = pw[k];
        if constexpr (!COLOUR) slots[i] = ps[k];
      }
    }
#pragma unroll
    for (int k = 0; k < KE; ++k) {
      const int el = tid + k * TPB;
      if (el < ne) {
#pragma unroll
        for (int a = 0; a < NLOC; ++a) {
          etab[el][a] = (pt[k][a] & kPtabIdMask) * RB;
          etab[el][NLOC + a] = (pt[k][a] >> kPtabLocalShift) * FB;
        }
        if constexpr (kGeoLds) {
          T g[16];
#pragma unroll
          for (int v = 0; v < 16 / GV; ++v)
#pragma unroll
            for (int t = 0; t < GV; ++t) g[v * GV + t] = pg[k][v].v[t];
#pragma unroll
          for (int i = 0; i < 12; ++i) geo[el][i] = g[i];
          const T sv0 = ORDER == 2 ? g[12] * T(0.05) : g[12];  // V / 20 (quadratic) or V (linear)
          geo[el][12] = g[13] * sv0;
          geo[el][13] = g[14] * sv0;
        }
      }
    }
    const int ce0 = e0, cne = ne, cnn = nn;
    __syncthreads();
    // B. the next patch's metadata
    const int pn = p + wx;
    // (and, when the geometry is read per work-item, the next patch's
    // element node words: the registers allow them across the element phase)
    constexpr bool kEarlyLate = !GEO;
    if (pn < stop) {
      fetch_meta(pn);
      if constexpr (kEarlyLate) fetch_late();
    }
    const int nj = spread_count<CW>(cne);
    const char* xb = reinterpret_cast<const char*>(x);
    char* fbase = reinterpret_cast<char*>(F);
#pragma unroll
    for (int pass = 0; pass < NP; ++pass) {
      const int c0 = pass * CW;
      // C. element phase of this pass
#pragma unroll
      for (int k = 0; k < KI; ++k) {
        const int w = tid + k * TPB;
        const int j = w / CW, r = w - j * CW;
        const int el = spread_element<CW>(j, cne);
        if (w >= nj * CW || el >= cne) continue;
        T Gm[4][3], clam, cmu;
        if constexpr (kGeoLds) {
#pragma unroll
          for (int kk = 0; kk < 4; ++kk)
#pragma unroll
            for (int d = 0; d < 3; ++d) Gm[kk][d] = geo[el][3 * kk + d];
          clam = geo[el][12];
          cmu = geo[el][13];
        } else {  // geometry row: G (12 values), volume, lambda, mu, as formed by the geometry kernel
          T g[16];
          const GR* row = reinterpret_cast<const GR*>(gcache + (int64_t(ce0) + el) * 16);
#pragma unroll
          for (int v = 0; v < 16 / GV; ++v) {
            const GR gv = row[v];
#pragma unroll
            for (int t = 0; t < GV; ++t) g[v * GV + t] = gv.v[t];
          }
#pragma unroll
          for (int kk = 0; kk < 4; ++kk)
#pragma unroll
            for (int d = 0; d < 3; ++d) Gm[kk][d] = g[3 * kk + d];
          const T sv0 = ORDER == 2 ? g[12] * T(0.05) : g[12];  // V / 20 (quadratic) or V (linear)
          clam = g[13] * sv0;
          cmu = g[14] * sv0;
        }
        uint32_t xo[NLOC], fo[NLOC];
        {
          const uint32_t rx = uint32_t(c0 + r) * uint32_t(sizeof(T)), rf = uint32_t(r) * 8u;
#pragma unroll
          for (int a = 0; a < NLOC; ++a) {
            xo[a] = etab[el][a] + rx;
            fo[a] = etab[el][NLOC + a] + rf;
          }
        }
        T en = T(0);
        auto u = [&](int a, int c) -> T {
          const T v = *reinterpret_cast<const T*>(xb + size_t(xo[a]) + size_t(c) * NR * sizeof(T));
          if constexpr (MASK) {
            const int32_t wd = words[(fo[a] - uint32_t(r) * 8u) / FB];
            return ((wd >> (kIdxBits + c)) & 1) ? T(0) : v;
          } else {
            return v;
          }
        };
        auto emit = [&](int a, const T f[3]) {
#pragma unroll
          for (int c = 0; c < 3; ++c)
            atomicAdd(reinterpret_cast<double*>(fbase + fo[a]) + c * CW, double(f[c]));
        };
        if constexpr (ORDER == 2) p2_apply<T>(Gm, clam, cmu, u, emit, GAMMA, en);
        else p1_apply<T>(Gm, clam, cmu, u, emit, GAMMA, en);
        if constexpr (GAMMA) {
          if constexpr (kLaneCase) en_acc[pass] += double(en);
          else atomicAdd(&gsum[c0 + r], double(en));
        }
      }
      // the next patch's metadata has arrived before this patch's write-back
      // stores are issued, so the next commit waits for no store (when the
      // element node words are fetched early)
      __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
      __syncthreads();
      // D. otherwise, the next patch's element node words now (in flight
      // during the write-back)
      if constexpr (!kEarlyLate) {
        if (pass == NP - 1 && pn < stop) fetch_late();
      }
      // E. write back this pass, zeroing F behind it.  Coloured form with
      // the geometry read per work-item, at 8 or more cases (at 4, FP64, it
      // measured 15% slower): the rows that are read, added to
      // and written back (nodes an earlier colour wrote, or y += K x) are all
      // read before the first store, so the reads do not wait for this
      // patch's stores (64^3 cube, 16 cases: 0.685 -> 0.669 ms FP32, 1.385 ->
      // 1.321 ms FP64).  The other forms read y only for y += K x and keep
      // one read per row piece, which measured faster for them; the
      // geometry-in-LDS variant has no registers to spare for it.  y is
      // written with streaming (non-temporal) stores: a product's y is
      // larger than the last-level cache at 16 cases, and keeping x there
      // instead measured faster (FP32 16 cases, bench.py's timing: coloured
      // 0.667-0.680 -> 0.651-0.669 ms, pipelined 0.703-0.706 -> 0.687-0.689).
      constexpr bool kReadFirst = COLOUR && !GEO && NR >= 8;
      V old[kReadFirst ? KIT : 1];
#pragma unroll
      for (int k = 0; k < (kReadFirst ? KIT : 0); ++k) {
        const int ent = sent + k * EPK;
        if (ent < cnn) {
          const int32_t wd = words[ent];
          const bool fixed = bc && ((wd >> (kIdxBits + sc)) & 1);
          if ((COLOUR || wd >= 0) && (add || (COLOUR && wd < 0)) && !fixed)
            old[k] = *reinterpret_cast<const V*>(y + size_t(wd & kIdxMask) * W + sc * NR + c0 + scc);
        }
      }
#pragma unroll
      for (int k = 0; k < KIT; ++k) {
        const int ent = sent + k * EPK;
        if (ent < cnn) {
          const int32_t wd = words[ent];
          const int col = sc * NR + c0 + scc;
          V v;
#pragma unroll
          for (int t = 0; t < VEC; ++t) {
            v.v[t] = T(F[ent * WC + sq + t]);
            F[ent * WC + sq + t] = 0.0;
          }
          const bool fixed = bc && ((wd >> (kIdxBits + sc)) & 1);
          if (!COLOUR && wd < 0) {  // shared node: partial sum to its staging slot
            T* sp = stage + size_t(slots[ent]) * W + col;
            if (stream) store_stream<T, VEC>(sp, v);
            else *reinterpret_cast<V*>(sp) = v;
          } else {
            V* yp = reinterpret_cast<V*>(y + size_t(wd & kIdxMask) * W + col);
            if (add || (COLOUR && wd < 0)) {  // y += (the caller, or an earlier colour, wrote y)
              if (!fixed) {  // (a fixed DOF keeps what y holds: the caller's value, or the first colour's zero)
                V o;
                if constexpr (kReadFirst) o = old[k];
                else o = *yp;
#pragma unroll
                for (int t = 0; t < VEC; ++t) o.v[t] += v.v[t];
                store_stream<T, VEC>(reinterpret_cast<T*>(yp), o);
              }
            } else {
              if (fixed) {
#pragma unroll
                for (int t = 0; t < VEC; ++t) v.v[t] = T(0);
              }
              store_stream<T, VEC>(reinterpret_cast<T*>(yp), v);
            }
          }
        }
      }
      __syncthreads();  // F (next pass), or words, slots, node tables and geometry (next patch)
    }
  }
  if constexpr (GAMMA) {
    if constexpr (kLaneCase) {
#pragma unroll
      for (int pass = 0; pass < NP; ++pass) {
        double v = en_acc[pass];
#pragma unroll
        for (int off = 32; off >= CW; off >>= 1) v += __shfl_xor(v, off, 64);
        if ((tid & 63) < CW) atomicAdd(&gsum[pass * CW + (tid & 63)], v);
      }
    }
    __syncthreads();
    fold_gamma<NR, TPB>(gsum, gamma, gslot, gcount);
  }
}

// as many persistent workgroups as fit on the device at once (measured
// occupancy x CUs), at most one per patch
template <typename T, int NR, int ORDER, bool MASK, bool GAMMA, bool COLOUR, bool GEO, int NP>
hipError_t launch_pipe_k(const ebe_mesh* m, const PatchLevel& L, const int32_t* plist, int64_t npatch, const void* x,
                         void* y, bool stream, bool bc, bool add, const int* gate, hipStream_t s, double* gamma) {
  constexpr int TPB = pipe_threads<T>(NR, ORDER, NP);
  static const int per_cu = [] {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_ebe_pipe<T, NR, ORDER, MASK, GAMMA, COLOUR, GEO, NP>, TPB,
                                                     0) != hipSuccess ||
        n < 1)
      n = 1;
    return n;
  }();
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, m->device) != hipSuccess || cus < 1)
    cus = 256;
  const int64_t grid = std::min<int64_t>(npatch, int64_t(per_cu) * cus);
  if (grid < 1) return hipSuccess;
  hipLaunchKernelGGL((k_ebe_pipe<T, NR, ORDER, MASK, GAMMA, COLOUR, GEO, NP>), dim3(unsigned(grid)), dim3(TPB), 0, s,
                     m->geo[sizeof(T) == 8 ? 0 : 1].as<T>(), L.ptab.as<uint32_t>(), L.pelem.as<int32_t>(),
                     L.poff.as<int32_t>(), COLOUR ? L.cword.as<int32_t>() : L.pnode.as<int32_t>(),
                     L.pslot.as<int32_t>(), plist, static_cast<const T*>(x), static_cast<T*>(y),
                     L.stage.as<T>(), int(stream), int(npatch), int(bc), int(add), gamma, m->gacc.as<double>(),
                     reinterpret_cast<unsigned*>(m->gacc.as<char>() + kGammaBytes - 64), gate);
  return hipGetLastError();
}

template <typename T, int NR, int ORDER, bool COLOUR, bool GEO, int NP>
hipError_t launch_pipe_c(const ebe_mesh* m, const PatchLevel& L, const int32_t* plist, int64_t npatch, const void* x,
                         void* y, bool stream, bool mask_in, bool bc, bool add, const int* gate, hipStream_t s,
                         double* gamma) {
  if (mask_in && gamma) return hipErrorInvalidValue;  // no caller needs both
  if (mask_in)
    return launch_pipe_k<T, NR, ORDER, true, false, COLOUR, GEO, NP>(m, L, plist, npatch, x, y, stream, bc, add,
                                                                    gate, s, nullptr);
  if (gamma)
    return launch_pipe_k<T, NR, ORDER, false, true, COLOUR, GEO, NP>(m, L, plist, npatch, x, y, stream, bc, add,
                                                                    gate, s, gamma);
  return launch_pipe_k<T, NR, ORDER, false, false, COLOUR, GEO, NP>(m, L, plist, npatch, x, y, stream, bc, add, gate,
                                                                   s, nullptr);
}

}  // namespace

template <typename T, int NR, int ORDER, bool GEO, int NP>
hipError_t launch_pipe(const ebe_mesh* m, const void* x, void* y, bool mask_in, bool bc, bool add, const int* gate,
                       hipStream_t s, double* gamma, bool colour) {
  const PatchLevel& L = m->pl[ORDER == 2 ? 0 : 1];
  if constexpr (ORDER == 2) {
    if (colour) {
      const int32_t* cp = L.cperm.as<int32_t>();
      for (size_t c = 0; c + 1 < L.coff.size(); ++c) {
        const hipError_t e = launch_pipe_c<T, NR, ORDER, true, GEO, NP>(
            m, L, cp + L.coff[c], L.coff[c + 1] - L.coff[c], x, y, false, mask_in, bc, add, gate, s, gamma);
        if (e != hipSuccess) return e;
      }
      return hipSuccess;
    }
  }
  if (colour) return hipErrorInvalidValue;
  // stream the staged partials past the caches when they cannot stay in the
  // last-level cache until the shared-node pass reads them back
  const bool st = int64_t(L.nslots) * 3 * NR * int64_t(sizeof(T)) > kStreamStageBytes;
  hipError_t e = launch_pipe_c<T, NR, ORDER, false, GEO, NP>(m, L, nullptr, L.npatch, x, y, st, mask_in, bc, add, gate,
                                                             s, gamma);
  if (e != hipSuccess || L.nshared == 0) return e;
  const int64_t work = L.nshared * (3 * NR / reduce_width<T, NR>());
  hipLaunchKernelGGL((k_reduce_shared<T, NR>), dim3(unsigned((work + 255) / 256)), dim3(256), 0, s,
                     L.snode.as<int32_t>(), L.soff.as<int32_t>(), L.stage.as<T>(), int(st), static_cast<T*>(y),
                     int32_t(L.nshared), int(bc), int(add), gate);
  return hipGetLastError();
}

}  // namespace ebe
