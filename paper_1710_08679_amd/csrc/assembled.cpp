// Host-side structure of the assembled operators: the sliced block layout
// (AsmOp) and level 2 of Algorithm 1(a), an algebraic coarsening of the
// linear (corner) mesh.
//
// The paper coarsens the first-order mesh algebraically for inner loop
// level 2 and stores the coarse matrix in 3x3 block rows (Section 2), but
// gives no coarsening.  Taken here: plain aggregation with one 3-DOF
// (translation) coarse node per aggregate, in three passes over the corners
// in increasing id on the corner graph:
//   1. a corner whose neighbours are all still free roots an aggregate made
//      of itself and its neighbours;
//   2. a corner still free joins the lowest-numbered aggregate among its
//      neighbours' pass-1 aggregates;
//   3. a corner still free (none: a corner left free by pass 1 had an
//      aggregated neighbour when it was visited) roots an aggregate with its
//      free neighbours.
// The tentative prolongator T copies coarse DOF (I, c) to DOF (a, c) of every
// member a that is not fixed; P2 = (I - omega D1^-1 K1p) T (smoothed
// aggregation: one damped block-Jacobi step on T, K1p = K1 without the fixed
// rows and columns, D1 its diagonal blocks with fixed DOFs set to identity),
// so fine row a of P2 reaches the aggregates of a's neighbours; A2 =
// P2^T K1p P2 (Galerkin) couples aggregates two steps apart.  Here: the
// structure of P2 (per fine row, its aggregates, increasing), of P2^T, and of
// A2's block rows; the values are formed on the GPU (setup_kernels.hip).
#include <algorithm>
#include <vector>

#include "ebe_internal.h"

namespace ebe {

namespace {

template <class T>
ebe_status up(DBuf& b, const std::vector<T>& h, hipStream_t s) {
  ebe_status st = b.alloc(std::max<size_t>(h.size(), 1) * sizeof(T));
  if (st != EBE_OK) return st;
  if (!h.empty())
    EBE_TRY_HIP(hipMemcpyAsync(b.as<void>(), h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
  return EBE_OK;
}

}  // namespace

ebe_status slice_rows(const std::vector<int32_t>& ptr, const std::vector<int32_t>& col, const uint8_t* fix,
                      std::vector<int32_t>& soff, std::vector<int32_t>& scol) {
  const int64_t n = int64_t(ptr.size()) - 1;
  const int64_t nsl = (n + kSliceRows - 1) / kSliceRows;
  soff.assign(nsl + 1, 0);
  for (int64_t sl = 0; sl < nsl; ++sl) {
    int32_t width = 0;
    for (int64_t v = sl * kSliceRows; v < std::min<int64_t>(n, (sl + 1) * kSliceRows); ++v)
      width = std::max(width, ptr[v + 1] - ptr[v]);
    if (int64_t(soff[sl]) + width >= (int64_t(1) << 31) / (9 * kSliceRows)) {
      set_error("assembled operator too large for 32-bit block indices");
      return EBE_ERR_ARG;
    }
    soff[sl + 1] = soff[sl] + width;
  }
  scol.assign(size_t(soff[nsl]) * kSliceRows, 0);
  for (int64_t v = 0; v < n; ++v) {
    const int64_t sl = v / kSliceRows, r = v - sl * kSliceRows;
    const int32_t len = ptr[v + 1] - ptr[v];
    for (int32_t j = 0; j < soff[sl + 1] - soff[sl]; ++j) {
      const int32_t c = j < len ? col[ptr[v] + j] : int32_t(v);
      scol[size_t(soff[sl] + j) * kSliceRows + r] = c | (int32_t(fix[c]) << kIdxBits);
    }
  }
  return EBE_OK;
}

ebe_status upload_asm(AsmOp& op, int64_t rows, const std::vector<int32_t>& soff, const std::vector<int32_t>& scol,
                      hipStream_t s) {
  ebe_status st = up(op.soff, soff, s);
  if (st == EBE_OK) st = up(op.col, scol, s);
  op.rows = rows;
  op.slots = soff.back();
  op.ready[0] = op.ready[1] = op.ready16 = false;
  return st;
}

ebe_status build_level2(ebe_mesh* m, const std::vector<int32_t>& bptr, const std::vector<int32_t>& bcol,
                        const uint8_t* fix, hipStream_t s) {
  const int64_t nv = int64_t(bptr.size()) - 1;
  // aggregation (the row of v in K1 is v and its neighbours)
  std::vector<int32_t> agg(nv, -1);
  int32_t na = 0;
  for (int64_t v = 0; v < nv; ++v) {  // pass 1
    if (agg[v] >= 0) continue;
    bool free = true;
    for (int32_t k = bptr[v]; k < bptr[v + 1] && free; ++k) free = agg[bcol[k]] < 0;
    if (!free) continue;
    for (int32_t k = bptr[v]; k < bptr[v + 1]; ++k) agg[bcol[k]] = na;
    ++na;
  }
  const std::vector<int32_t> first(agg);
  for (int64_t v = 0; v < nv; ++v) {  // pass 2
    if (first[v] >= 0) continue;
    int32_t best = -1;
    for (int32_t k = bptr[v]; k < bptr[v + 1]; ++k) {
      const int32_t a = first[bcol[k]];
      if (a >= 0 && (best < 0 || a < best)) best = a;
    }
    agg[v] = best;
  }
  for (int64_t v = 0; v < nv; ++v) {  // pass 3
    if (agg[v] >= 0) continue;
    for (int32_t k = bptr[v]; k < bptr[v + 1]; ++k)
      if (agg[bcol[k]] < 0) agg[bcol[k]] = na;
    ++na;
  }
  // coarse fix bits: a component is fixed when it is fixed at every member
  std::vector<uint8_t> cfix(na, 7);
  for (int64_t v = 0; v < nv; ++v) cfix[agg[v]] &= uint8_t(fix[v] & 7);
  // P2 rows: the aggregates of v and its neighbours, increasing, padded with -1
  int32_t width = 1;
  std::vector<int32_t> tmp;
  for (int64_t v = 0; v < nv; ++v) {
    tmp.clear();
    for (int32_t k = bptr[v]; k < bptr[v + 1]; ++k) tmp.push_back(agg[bcol[k]]);
    std::sort(tmp.begin(), tmp.end());
    width = std::max(width, int32_t(std::unique(tmp.begin(), tmp.end()) - tmp.begin()));
  }
  std::vector<int32_t> pcol(size_t(nv) * width, -1);
  for (int64_t v = 0; v < nv; ++v) {
    tmp.clear();
    for (int32_t k = bptr[v]; k < bptr[v + 1]; ++k) tmp.push_back(agg[bcol[k]]);
    std::sort(tmp.begin(), tmp.end());
    tmp.erase(std::unique(tmp.begin(), tmp.end()), tmp.end());
    std::copy(tmp.begin(), tmp.end(), pcol.begin() + size_t(v) * width);
  }
  if (int64_t(nv) * width >= (int64_t(1) << 31) / 9) {
    set_error("level 2: prolongator too large for 32-bit indices");
    return EBE_ERR_ARG;
  }
  // P2^T: for each aggregate, the P2 entries (v * width + w) naming it, in v order
  std::vector<int32_t> toff(na + 1, 0), tidx;
  for (size_t i = 0; i < pcol.size(); ++i)
    if (pcol[i] >= 0) toff[pcol[i] + 1]++;
  for (int32_t a = 0; a < na; ++a) toff[a + 1] += toff[a];
  tidx.resize(toff[na]);
  {
    std::vector<int32_t> fill(toff.begin(), toff.end() - 1);
    for (size_t i = 0; i < pcol.size(); ++i)
      if (pcol[i] >= 0) tidx[fill[pcol[i]]++] = int32_t(i);
  }
  // A2 rows: J reached from I through P2^T, K1 and P2, increasing
  std::vector<int32_t> aptr(na + 1, 0), acol, alen(na);
  std::vector<int32_t> stamp(na, -1);
  for (int32_t a = 0; a < na; ++a) {
    const size_t b0 = acol.size();
    for (int32_t t = toff[a]; t < toff[a + 1]; ++t) {
      const int64_t v = tidx[t] / width;
      for (int32_t k = bptr[v]; k < bptr[v + 1]; ++k) {
        const int32_t* pr = pcol.data() + size_t(bcol[k]) * width;
        for (int32_t w = 0; w < width && pr[w] >= 0; ++w)
          if (stamp[pr[w]] != a) {
            stamp[pr[w]] = a;
            acol.push_back(pr[w]);
          }
      }
    }
    std::sort(acol.begin() + b0, acol.end());
    aptr[a + 1] = int32_t(acol.size());
    alen[a] = aptr[a + 1] - aptr[a];
  }
  std::vector<int32_t> asoff, ascol;
  ebe_status st = slice_rows(aptr, acol, cfix.data(), asoff, ascol);
  if (st != EBE_OK) return st;
  m->n_agg = na;
  m->p2_width = width;
  m->a2_maxlen = alen.empty() ? 0 : *std::max_element(alen.begin(), alen.end());

  if ((st = up(m->agg, agg, s)) != EBE_OK) return st;
  if ((st = up(m->cfix, cfix, s)) != EBE_OK) return st;
  if ((st = up(m->p2_col, pcol, s)) != EBE_OK) return st;
  if ((st = up(m->p2t_off, toff, s)) != EBE_OK) return st;
  if ((st = up(m->p2t_idx, tidx, s)) != EBE_OK) return st;
  if ((st = up(m->a2_len, alen, s)) != EBE_OK) return st;
  return upload_asm(m->a2, na, asoff, ascol, s);
}

}  // namespace ebe
