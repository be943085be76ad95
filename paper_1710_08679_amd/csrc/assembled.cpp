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
// P2 copies coarse DOF (I, c) to DOF (a, c) of every member a that is not
// fixed; A2 = P2^T K1 P2 (Galerkin), so its block (I, J) is the sum of the
// K1 blocks (a, b), a in I, b in J, with fixed rows and columns left out.
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
  op.ready[0] = op.ready[1] = false;
  return st;
}

ebe_status build_level2(ebe_mesh* m, const std::vector<int32_t>& bptr, const std::vector<int32_t>& bcol,
                        const std::vector<int32_t>& k1soff, const uint8_t* fix, hipStream_t s) {
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
  // members (increasing) and coarse fix bits
  std::vector<int32_t> moff(na + 1, 0), mem(nv);
  for (int64_t v = 0; v < nv; ++v) moff[agg[v] + 1]++;
  for (int32_t a = 0; a < na; ++a) moff[a + 1] += moff[a];
  {
    std::vector<int32_t> fill(moff.begin(), moff.end() - 1);
    for (int64_t v = 0; v < nv; ++v) mem[fill[agg[v]]++] = int32_t(v);
  }
  std::vector<uint8_t> cfix(na, 7);
  for (int64_t v = 0; v < nv; ++v) cfix[agg[v]] &= uint8_t(fix[v] & 7);
  // A2 rows: the aggregates of the members' neighbours, increasing
  std::vector<int32_t> aptr(na + 1, 0), acol;
  std::vector<int32_t> stamp(na, -1);
  for (int32_t a = 0; a < na; ++a) {
    const size_t b0 = acol.size();
    for (int32_t i = moff[a]; i < moff[a + 1]; ++i) {
      const int32_t v = mem[i];
      for (int32_t k = bptr[v]; k < bptr[v + 1]; ++k) {
        const int32_t b = agg[bcol[k]];
        if (stamp[b] != a) {
          stamp[b] = a;
          acol.push_back(b);
        }
      }
    }
    std::sort(acol.begin() + b0, acol.end());
    aptr[a + 1] = int32_t(acol.size());
  }
  std::vector<int32_t> asoff, ascol;
  ebe_status st = slice_rows(aptr, acol, cfix.data(), asoff, ascol);
  if (st != EBE_OK) return st;
  // for each K1 entry, the A2 entry its block adds into
  std::vector<int32_t> map(size_t(k1soff.back()) * kSliceRows, -1);
  for (int64_t v = 0; v < nv; ++v) {
    const int64_t sl = v / kSliceRows, r = v - sl * kSliceRows;
    const int32_t I = agg[v];
    const int64_t sI = I / kSliceRows, rI = I - sI * kSliceRows;
    for (int32_t j = 0; j < bptr[v + 1] - bptr[v]; ++j) {
      const int32_t J = agg[bcol[bptr[v] + j]];
      const int32_t jj = int32_t(std::lower_bound(acol.begin() + aptr[I], acol.begin() + aptr[I + 1], J) -
                                 (acol.begin() + aptr[I]));
      map[size_t(k1soff[sl] + j) * kSliceRows + r] = int32_t((asoff[sI] + jj) * kSliceRows + rI);
    }
  }
  m->n_agg = na;
  if ((st = up(m->agg, agg, s)) != EBE_OK) return st;
  if ((st = up(m->mem_off, moff, s)) != EBE_OK) return st;
  if ((st = up(m->mem, mem, s)) != EBE_OK) return st;
  if ((st = up(m->cfix, cfix, s)) != EBE_OK) return st;
  if ((st = up(m->a2_map, map, s)) != EBE_OK) return st;
  return upload_asm(m->a2, na, asoff, ascol, s);
}

}  // namespace ebe
