// Element patches: the work decomposition of the EBE products.
//
// Elements are cut, in the order given, into patches of at most kPatchElems
// elements touching at most kPatchNodes distinct nodes.  A workgroup owns one
// patch: it accumulates the patch's element forces in LDS, then writes each
// patch node once.  A node touched by a single patch ("exclusive") is written
// straight to the output; a node touched by several patches ("shared") gets
// one partial sum per patch in a staging buffer, and a second, node-centric
// pass adds those partials in patch order.  No atomics reach global memory
// and the result does not depend on scheduling.
//
// The linear level (corner nodes only) has patches of its own, larger in
// elements: a linear element's product is a fraction of a quadratic one's,
// so its workgroups need more elements to carry the fixed cost of a patch.
#include <algorithm>
#include <cstring>
#include <vector>

#include "ebe_internal.h"

namespace ebe {

namespace {

struct LevelTables {
  std::vector<int32_t> poff, pnode, pslot;      // per patch entries
  std::vector<int32_t> snode, soff;             // reduction of shared nodes
  int64_t nslots = 0;
  int max_nodes = 0;
};

// Entries of one level: nodes_of(e, a) for local slot a < nloc.
template <class NodeOf>
void build_level(const std::vector<int32_t>& pelem, int nloc, int64_t n_nodes, const uint8_t* fix,
                 NodeOf node_of, std::vector<uint8_t>& lconn, int lstride, LevelTables& t) {
  const int64_t npatch = int64_t(pelem.size()) - 1;
  std::vector<int32_t> stamp(n_nodes, -1), local(n_nodes, 0), count(n_nodes, 0);
  t.poff.assign(npatch + 1, 0);
  t.pnode.clear();
  for (int64_t p = 0; p < npatch; ++p) {
    const int32_t base = int32_t(t.pnode.size());
    for (int32_t e = pelem[p]; e < pelem[p + 1]; ++e) {
      for (int a = 0; a < nloc; ++a) {
        const int32_t v = node_of(e, a);
        if (stamp[v] != int32_t(p)) {
          stamp[v] = int32_t(p);
          local[v] = int32_t(t.pnode.size()) - base;
          t.pnode.push_back(v);
          count[v]++;
        }
        lconn[size_t(e) * lstride + a] = uint8_t(local[v]);
      }
    }
    t.poff[p + 1] = int32_t(t.pnode.size());
    t.max_nodes = std::max(t.max_nodes, t.poff[p + 1] - base);
  }
  // Staging slots: the partial sums of one shared node sit in consecutive
  // slots, nodes in increasing id, a node's partials in patch order.  start[]
  // is cumulative over shared nodes only, so it doubles as the offset list.
  std::vector<int64_t> start(n_nodes + 1, 0);
  for (int64_t v = 0; v < n_nodes; ++v) start[v + 1] = start[v] + (count[v] > 1 ? count[v] : 0);
  t.nslots = start[n_nodes];
  t.pslot.assign(t.pnode.size(), -1);
  std::vector<int64_t> fill(start.begin(), start.end() - 1);
  for (size_t i = 0; i < t.pnode.size(); ++i) {
    const int32_t v = t.pnode[i];
    if (count[v] > 1) t.pslot[i] = int32_t(fill[v]++);
  }
  t.snode.clear();
  t.soff.assign(1, 0);
  for (int64_t v = 0; v < n_nodes; ++v)
    if (count[v] > 1) {
      t.snode.push_back(int32_t(v) | (int32_t(fix[v]) << kIdxBits));
      t.soff.push_back(int32_t(start[v + 1]));
    }
  // pack node words: id | fix bits | shared flag
  for (size_t i = 0; i < t.pnode.size(); ++i) {
    const int32_t v = t.pnode[i];
    t.pnode[i] = v | (int32_t(fix[v]) << kIdxBits) | (count[v] > 1 ? int32_t(1u << 31) : 0);
  }
}

// Cut elements, in order, into ranges of at most max_elems elements touching
// at most max_nodes distinct nodes (the nloc nodes of element e are
// node_of(e, 0..nloc-1), distinct within an element).
template <class NodeOf>
std::vector<int32_t> cut_patches(int64_t E, int nloc, int64_t n_nodes, int max_elems, int max_nodes,
                                 NodeOf node_of) {
  std::vector<int32_t> pelem(1, 0), stamp(n_nodes, -1);
  int32_t pid = 0, ne = 0, nn = 0;
  for (int64_t e = 0; e < E; ++e) {
    int fresh = 0;
    for (int a = 0; a < nloc; ++a) fresh += stamp[node_of(e, a)] != pid;
    if (ne == max_elems || nn + fresh > max_nodes) {
      pelem.push_back(int32_t(e));
      ++pid;
      ne = 0;
      nn = 0;
    }
    for (int a = 0; a < nloc; ++a) {
      const int32_t v = node_of(e, a);
      if (stamp[v] != pid) {
        stamp[v] = pid;
        ++nn;
      }
    }
    ++ne;
  }
  pelem.push_back(int32_t(E));
  return pelem;
}

// Element node words: node id | patch-local id << kPtabLocalShift, [E][nloc].
template <class NodeOf>
std::vector<uint32_t> node_words(int64_t E, int nloc, NodeOf node_of, const std::vector<uint8_t>& lconn,
                                 int lstride) {
  std::vector<uint32_t> w(size_t(E) * nloc);
  for (int64_t e = 0; e < E; ++e)
    for (int a = 0; a < nloc; ++a)
      w[size_t(e) * nloc + a] =
          uint32_t(node_of(e, a)) | (uint32_t(lconn[size_t(e) * lstride + a]) << kPtabLocalShift);
  return w;
}

// Greedy colouring of the patches (in patch order, each takes the smallest
// colour no patch sharing a node with it has), the patches listed colour by
// colour, and the node words with bit 31 set where an earlier patch in that
// order already wrote the node.
void colour_patches(int64_t n_nodes, const LevelTables& t, std::vector<int32_t>& cperm, std::vector<int64_t>& coff,
                    std::vector<int32_t>& cword) {
  const int64_t npatch = int64_t(t.poff.size()) - 1;
  // node -> patches (CSR)
  std::vector<int32_t> nstart(n_nodes + 1, 0);
  for (int32_t w : t.pnode) nstart[(w & kIdxMask) + 1]++;
  for (int64_t v = 0; v < n_nodes; ++v) nstart[v + 1] += nstart[v];
  std::vector<int32_t> npatches(t.pnode.size()), fillp(nstart.begin(), nstart.end() - 1);
  for (int64_t p = 0; p < npatch; ++p)
    for (int32_t i = t.poff[p]; i < t.poff[p + 1]; ++i) npatches[fillp[t.pnode[i] & kIdxMask]++] = int32_t(p);
  std::vector<int32_t> colour(npatch, -1);
  std::vector<int64_t> taken;  // taken[c] == p: colour c is used by a neighbour of patch p
  int ncol = 0;
  for (int64_t p = 0; p < npatch; ++p) {
    for (int32_t i = t.poff[p]; i < t.poff[p + 1]; ++i) {
      const int32_t v = t.pnode[i] & kIdxMask;
      for (int32_t k = nstart[v]; k < nstart[v + 1]; ++k) {
        const int32_t c = colour[npatches[k]];
        if (c >= 0) taken[c] = p;
      }
    }
    int c = 0;
    while (c < ncol && taken[c] == p) ++c;
    if (c == ncol) {
      ++ncol;
      taken.push_back(-1);
    }
    colour[p] = c;
  }
  coff.assign(ncol + 1, 0);
  for (int64_t p = 0; p < npatch; ++p) coff[colour[p] + 1]++;
  for (int c = 0; c < ncol; ++c) coff[c + 1] += coff[c];
  cperm.assign(npatch, 0);
  std::vector<int64_t> fillc(coff.begin(), coff.end() - 1);
  for (int64_t p = 0; p < npatch; ++p) cperm[fillc[colour[p]]++] = int32_t(p);
  cword.assign(t.pnode.size(), 0);
  std::vector<uint8_t> written(n_nodes, 0);
  for (int64_t k = 0; k < npatch; ++k) {
    const int32_t p = cperm[k];
    for (int32_t i = t.poff[p]; i < t.poff[p + 1]; ++i) {
      const int32_t w = t.pnode[i] & 0x7fffffff;  // id | fix bits
      const int32_t v = w & kIdxMask;
      cword[i] = w | (written[v] ? int32_t(1u << 31) : 0);
      written[v] = 1;
    }
  }
}

template <class T>
ebe_status up(DBuf& b, const std::vector<T>& h, hipStream_t s) {
  ebe_status st = b.alloc(std::max<size_t>(h.size(), 1) * sizeof(T));
  if (st != EBE_OK) return st;
  if (!h.empty())
    EBE_TRY_HIP(hipMemcpyAsync(b.as<void>(), h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
  return EBE_OK;
}

}  // namespace

ebe_status build_patches(ebe_mesh* m, const int32_t* conn10, const uint8_t* fix, hipStream_t s) {
  const int64_t E = m->n_elem;
  auto node_of = [&](int64_t e, int a) { return conn10[size_t(e) * 10 + a]; };
  // 1. cut elements into patches, separately for each level
  std::vector<int32_t> pelem[2] = {cut_patches(E, 10, m->n_nodes, kPatchElems, kPatchNodes, node_of),
                                   cut_patches(E, 4, m->n_vertices, kLinPatchElems, kLinPatchCorners, node_of)};
  // 2. quadratic level (all 10 nodes) and linear level (corners)
  std::vector<uint8_t> lconn(size_t(E) * 16, 0), lconn1(size_t(E) * 4, 0);
  LevelTables t[2];
  build_level(pelem[0], 10, m->n_nodes, fix, node_of, lconn, 16, t[0]);
  build_level(pelem[1], 4, m->n_vertices, fix, node_of, lconn1, 4, t[1]);
  if (t[0].max_nodes > kPatchNodes || t[1].max_nodes > kLinPatchCorners) {
    set_error("build_patches: patch with %d nodes / %d corners exceeds %d / %d", t[0].max_nodes, t[1].max_nodes,
              kPatchNodes, kLinPatchCorners);
    return EBE_ERR_INDEX;
  }
  ebe_status st = EBE_OK;
  if ((st = up(m->lconn, lconn, s)) != EBE_OK) return st;
  if ((st = up(m->lconn1, lconn1, s)) != EBE_OK) return st;
  if (m->n_nodes <= int64_t(kPtabIdMask)) {  // element node words (pipelined and coloured forms)
    if ((st = up(m->pl[0].ptab, node_words(E, 10, node_of, lconn, 16), s)) != EBE_OK) return st;
    if ((st = up(m->pl[1].ptab, node_words(E, 4, node_of, lconn1, 4), s)) != EBE_OK) return st;
  }
  {
    std::vector<int32_t> cperm, cword;
    colour_patches(m->n_nodes, t[0], cperm, m->pl[0].coff, cword);
    if ((st = up(m->pl[0].cperm, cperm, s)) != EBE_OK) return st;
    if ((st = up(m->pl[0].cword, cword, s)) != EBE_OK) return st;
  }
  {
    // incidence lists of the quadratic patches: for each patch entry, the
    // element slots that touch it, in element order (deterministic form)
    const std::vector<int32_t>& pe = pelem[0];
    const LevelTables& t0 = t[0];
    std::vector<uint16_t> pinc(size_t(E) * 10);
    std::vector<int32_t> pistart(t0.pnode.size());
    std::vector<int32_t> cnt;
    for (size_t p = 0; p + 1 < pe.size(); ++p) {
      const int32_t e0 = pe[p], ne = pe[p + 1] - e0, o0 = t0.poff[p], nn = t0.poff[p + 1] - o0;
      cnt.assign(size_t(nn) + 1, 0);
      for (int32_t el = 0; el < ne; ++el)
        for (int a = 0; a < 10; ++a) cnt[lconn[(size_t(e0) + el) * 16 + a] + 1]++;
      for (int32_t i = 0; i < nn; ++i) cnt[i + 1] += cnt[i];
      for (int32_t i = 0; i < nn; ++i) pistart[size_t(o0) + i] = cnt[i];
      for (int32_t el = 0; el < ne; ++el)
        for (int a = 0; a < 10; ++a) {
          const int lid = lconn[(size_t(e0) + el) * 16 + a];
          pinc[size_t(e0) * 10 + cnt[lid]++] = uint16_t(el * 10 + a);
        }
    }
    if ((st = up(m->pl[0].pinc, pinc, s)) != EBE_OK) return st;
    if ((st = up(m->pl[0].pistart, pistart, s)) != EBE_OK) return st;
  }
  for (int l = 0; l < 2; ++l) {
    PatchLevel& L = m->pl[l];
    if ((st = up(L.pelem, pelem[l], s)) != EBE_OK) return st;
    if ((st = up(L.poff, t[l].poff, s)) != EBE_OK) return st;
    if ((st = up(L.pnode, t[l].pnode, s)) != EBE_OK) return st;
    if ((st = up(L.pslot, t[l].pslot, s)) != EBE_OK) return st;
    if ((st = up(L.snode, t[l].snode, s)) != EBE_OK) return st;
    if ((st = up(L.soff, t[l].soff, s)) != EBE_OK) return st;
    L.npatch = int64_t(pelem[l].size()) - 1;
    L.nslots = t[l].nslots;
    L.nshared = int64_t(t[l].snode.size());
    L.entries = int64_t(t[l].pnode.size());
    L.max_nodes = t[l].max_nodes;
  }
  return EBE_OK;
}

}  // namespace ebe
