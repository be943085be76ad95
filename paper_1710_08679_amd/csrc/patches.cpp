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
// The same patches serve the linear level, restricted to corner nodes.
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
  // 1. cut elements into patches
  std::vector<int32_t> pelem(1, 0);
  {
    std::vector<int32_t> stamp(m->n_nodes, -1);
    int32_t pid = 0, ne = 0, nn = 0, nc = 0;
    for (int64_t e = 0; e < E; ++e) {
      const int32_t* c = conn10 + 10 * e;
      int fresh = 0, fresh_c = 0;  // nodes (corners) of e not yet in the patch (an element's nodes are distinct)
      for (int a = 0; a < 10; ++a)
        if (stamp[c[a]] != pid) {
          ++fresh;
          if (a < 4) ++fresh_c;
        }
      if (ne == kPatchElems || nn + fresh > kPatchNodes || nc + fresh_c > kPatchCorners) {
        pelem.push_back(int32_t(e));
        ++pid;
        ne = 0;
        nn = 0;
        nc = 0;
      }
      for (int a = 0; a < 10; ++a)
        if (stamp[c[a]] != pid) {
          stamp[c[a]] = pid;
          ++nn;
          if (a < 4) ++nc;
        }
      ++ne;
    }
    pelem.push_back(int32_t(E));
  }
  m->n_patch = int64_t(pelem.size()) - 1;

  // 2. quadratic level (all 10 nodes) and linear level (corners)
  std::vector<uint8_t> lconn(size_t(E) * 16, 0), lconn1(size_t(E) * 4, 0);
  LevelTables t2, t1;
  build_level(pelem, 10, m->n_nodes, fix, [&](int32_t e, int a) { return conn10[size_t(e) * 10 + a]; }, lconn, 16,
              t2);
  build_level(pelem, 4, m->n_vertices, fix, [&](int32_t e, int a) { return conn10[size_t(e) * 10 + a]; }, lconn1,
              4, t1);
  if (t2.max_nodes > kPatchNodes || t1.max_nodes > kPatchCorners) {
    set_error("build_patches: patch with %d nodes / %d corners exceeds %d / %d", t2.max_nodes, t1.max_nodes,
              kPatchNodes, kPatchCorners);
    return EBE_ERR_INDEX;
  }
  ebe_status st = EBE_OK;
  PatchLevel* L[2] = {&m->pl[0], &m->pl[1]};
  LevelTables* T[2] = {&t2, &t1};
  if ((st = up(m->pelem, pelem, s)) != EBE_OK) return st;
  if ((st = up(m->lconn, lconn, s)) != EBE_OK) return st;
  if ((st = up(m->lconn1, lconn1, s)) != EBE_OK) return st;
  for (int l = 0; l < 2; ++l) {
    if ((st = up(L[l]->poff, T[l]->poff, s)) != EBE_OK) return st;
    if ((st = up(L[l]->pnode, T[l]->pnode, s)) != EBE_OK) return st;
    if ((st = up(L[l]->pslot, T[l]->pslot, s)) != EBE_OK) return st;
    if ((st = up(L[l]->snode, T[l]->snode, s)) != EBE_OK) return st;
    if ((st = up(L[l]->soff, T[l]->soff, s)) != EBE_OK) return st;
    L[l]->nslots = T[l]->nslots;
    L[l]->nshared = int64_t(T[l]->snode.size());
    L[l]->entries = int64_t(T[l]->pnode.size());
    L[l]->max_nodes = T[l]->max_nodes;
  }
  return EBE_OK;
}

}  // namespace ebe
