// Batches of meshes, each with its own set of cases.  Section 5 solves its
// 368 cases as 23 sets of 16, one set after another; a batch instead keeps
// the GPU full with many solves at once, in two ways:
//
// Merged groups.  Meshes of at most `merge_elems` elements (too small to
// fill the GPU alone) are grouped by case count (bands (8,16], (4,8], (2,4],
// [1,2]) into block-diagonal merged meshes of at most kGroupElems elements,
// built once (on the first solve) from the members' device copies: member
// nodes renumbered vertex-first into one mesh, their elements one after the
// other.  A merged mesh's patches are the members' patches, so every product
// and vector pass of its solve is one launch over the (member, patch) work
// list of all members, and its inner loops replay as captured HIP graphs.
// Each member's cases are the merged system's first cases, scaled to unit
// norm (a zero case stays zero), and the merged solve runs to tol / sqrt(m)
// for m members: the merged relative residual of a case is then at most tol
// only if every member's is, since the squared residual norms add up over
// the members.  After the solve each member's displacement is unscaled and
// its own residual ||P(f - K u)|| / ||P f|| is formed with its own operator
// for the statistics.
//
// Lanes.  Merged groups and the remaining (larger) meshes are solved by up
// to kLanes worker threads, each with its own stream (default priority),
// largest job first; the solver synchronises only its own stream, so the
// kernels of different jobs overlap on the GPU's hardware queues.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <new>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "batch_kernels.h"
#include "ebe_internal.h"

using namespace ebe;

namespace {
constexpr int kLanes = 4;                          // concurrent jobs: one per hardware queue a process gets by default
// merging is off unless asked for (ebe_batch_set_merge): on the 32 + 1 mesh
// serving set it measured slower than concurrent solves alone (3.03 s with
// meshes <= 150k elements merged, 4.70 s with meshes <= 600k merged into
// groups of <= 4M, against 2.77 s): every member iterates until the hardest
// one converges, to a tolerance sqrt(members) tighter, on cases padded to
// the group's largest count, and large merged jobs balance worse over the
// worker streams
constexpr int64_t kDefaultMergeElems = 0;
constexpr int64_t kGroupElems = 1000000;           // elements of one merged mesh, at most

struct Group {
  std::vector<int32_t> members;  // batch indices, in merged order
  int32_t nr = 0;                // cases of the merged system (the largest member's)
  ebe_mesh* mesh = nullptr;      // merged mesh (owned)
  std::vector<std::unique_ptr<DBuf>> maps;  // per member: int32 [N_i] merged node ids
  DBuf F, U;                     // merged load and solution [N][3][nr]
  DBuf scale;                    // double [members][EBE_MAX_RHS]
  DBuf norms;                    // double [2 EBE_MAX_RHS]
  DBuf tmp;                      // a member's K u [N_i][3][n_i], largest member
  ~Group() { ebe_mesh_destroy(mesh); }
};

int band_of(int32_t n) { return n > 8 ? 0 : (n > 4 ? 1 : (n > 2 ? 2 : 3)); }

template <class T>
ebe_status d2h(std::vector<T>& out, const DBuf& b, size_t count) {
  out.resize(count);
  if (count) EBE_TRY_HIP(hipMemcpy(out.data(), b.as<void>(), count * sizeof(T), hipMemcpyDeviceToHost));
  return EBE_OK;
}

// The merged mesh of g.members (host arrays rebuilt from the members' device
// copies: corner coordinates, edge ends, connectivity, moduli, fix bits).
ebe_status build_group(const std::vector<ebe_mesh*>& meshes, Group& g, hipStream_t s) {
  int64_t Nv = 0, Ne = 0, E = 0;
  for (int32_t i : g.members) {
    Nv += meshes[i]->n_vertices;
    Ne += meshes[i]->n_nodes - meshes[i]->n_vertices;
    E += meshes[i]->n_elem;
  }
  const int64_t N = Nv + Ne;
  std::vector<double> xyz(size_t(N) * 3), young(E), poisson(E);
  std::vector<int32_t> conn(size_t(E) * 10);
  std::vector<uint8_t> fixed(size_t(N) * 3, 0);
  bool any_fixed = false;
  int64_t voff = 0, eoff = 0, el0 = 0;
  for (int32_t i : g.members) {
    const ebe_mesh* m = meshes[i];
    const int64_t Ni = m->n_nodes, Nvi = m->n_vertices, Ei = m->n_elem;
    std::vector<double4> xv;
    std::vector<int32_t> ends, ci;
    std::vector<double> yi, pi;
    std::vector<uint8_t> fi;
    ebe_status st = d2h(xv, m->xv, size_t(Nvi));
    if (st == EBE_OK) st = d2h(ends, m->edge_ends, size_t(Ni - Nvi) * 2);
    if (st == EBE_OK) st = d2h(ci, m->conn, size_t(Ei) * 10);
    if (st == EBE_OK) st = d2h(yi, m->young, size_t(Ei));
    if (st == EBE_OK) st = d2h(pi, m->poisson, size_t(Ei));
    if (st == EBE_OK) st = d2h(fi, m->fix, size_t(Ni));
    if (st != EBE_OK) return st;
    std::vector<int32_t> map(Ni);
    for (int64_t v = 0; v < Ni; ++v) map[v] = int32_t(v < Nvi ? voff + v : Nv + eoff + (v - Nvi));
    for (int64_t v = 0; v < Ni; ++v) {
      double* x = &xyz[size_t(map[v]) * 3];
      if (v < Nvi) {
        x[0] = xv[v].x;
        x[1] = xv[v].y;
        x[2] = xv[v].z;
      } else {  // edge nodes sit at their edge's midpoint (checked when the member was created)
        const double4 a = xv[ends[2 * (v - Nvi)]], b = xv[ends[2 * (v - Nvi) + 1]];
        x[0] = 0.5 * (a.x + b.x);
        x[1] = 0.5 * (a.y + b.y);
        x[2] = 0.5 * (a.z + b.z);
      }
      for (int c = 0; c < 3; ++c) {
        fixed[size_t(map[v]) * 3 + c] = (fi[v] >> c) & 1;
        any_fixed |= ((fi[v] >> c) & 1) != 0;
      }
    }
    for (int64_t k = 0; k < Ei * 10; ++k) conn[size_t(el0) * 10 + k] = map[ci[k] & kIdxMask];
    std::copy(yi.begin(), yi.end(), young.begin() + el0);
    std::copy(pi.begin(), pi.end(), poisson.begin() + el0);
    auto dm = std::make_unique<DBuf>();
    if ((st = dm->alloc(size_t(Ni) * sizeof(int32_t))) != EBE_OK) return st;
    EBE_TRY_HIP(hipMemcpy(dm->as<void>(), map.data(), size_t(Ni) * sizeof(int32_t), hipMemcpyHostToDevice));
    g.maps.push_back(std::move(dm));
    voff += Nvi;
    eoff += Ni - Nvi;
    el0 += Ei;
  }
  ebe_status st = ebe_mesh_create(xyz.data(), N, Nv, conn.data(), E, young.data(), poisson.data(),
                                  any_fixed ? fixed.data() : nullptr, s, &g.mesh);
  if (st != EBE_OK) return st;
  int64_t tmp = 0;
  for (int32_t i : g.members) tmp = std::max<int64_t>(tmp, meshes[i]->n_nodes * 3 * EBE_MAX_RHS);
  const size_t vb = size_t(N) * 3 * g.nr * sizeof(double);
  if ((st = g.F.alloc(vb)) != EBE_OK || (st = g.U.alloc(vb)) != EBE_OK) return st;
  if ((st = g.scale.alloc(g.members.size() * EBE_MAX_RHS * sizeof(double))) != EBE_OK) return st;
  if ((st = g.norms.alloc(2 * EBE_MAX_RHS * sizeof(double))) != EBE_OK) return st;
  return g.tmp.alloc(size_t(tmp) * sizeof(double));
}

}  // namespace

struct ebe_batch {
  std::vector<ebe_mesh*> meshes;
  std::vector<int32_t> nrhs;
  std::vector<hipStream_t> lanes;  // worker streams
  int device = 0;
  int64_t merge_elems = kDefaultMergeElems;
  bool planned = false;
  std::vector<std::unique_ptr<Group>> groups;
  std::vector<int32_t> solo;  // meshes solved on their own
};

namespace {

// Group the small meshes (once per batch, on the first solve).
ebe_status plan(ebe_batch* b, hipStream_t s) {
  b->groups.clear();
  b->solo.clear();
  const int32_t n = int32_t(b->meshes.size());
  std::vector<int32_t> small[4];
  for (int32_t i = 0; i < n; ++i) {
    // curved meshes are solved on their own (the merged mesh is built straight-sided)
    if (b->merge_elems > 0 && b->meshes[i]->n_elem <= b->merge_elems && !b->meshes[i]->curved)
      small[band_of(b->nrhs[i])].push_back(i);
    else b->solo.push_back(i);
  }
  for (auto& band : small) {
    // largest case count first, then larger meshes first
    std::stable_sort(band.begin(), band.end(), [&](int32_t a, int32_t c) {
      return b->nrhs[a] != b->nrhs[c] ? b->nrhs[a] > b->nrhs[c] : b->meshes[a]->n_elem > b->meshes[c]->n_elem;
    });
    std::vector<int32_t> cur;
    int64_t elems = 0;
    auto flush = [&]() -> ebe_status {
      if (cur.size() == 1) b->solo.push_back(cur[0]);
      if (cur.size() >= 2) {
        auto g = std::make_unique<Group>();
        g->members = cur;
        for (int32_t i : cur) g->nr = std::max(g->nr, b->nrhs[i]);
        ebe_status st = build_group(b->meshes, *g, s);
        if (st != EBE_OK) return st;
        b->groups.push_back(std::move(g));
      }
      cur.clear();
      elems = 0;
      return EBE_OK;
    };
    for (int32_t i : band) {
      if (!cur.empty() && elems + b->meshes[i]->n_elem > kGroupElems) {
        ebe_status st = flush();
        if (st != EBE_OK) return st;
      }
      cur.push_back(i);
      elems += b->meshes[i]->n_elem;
    }
    ebe_status st = flush();
    if (st != EBE_OK) return st;
  }
  b->planned = true;
  return EBE_OK;
}

// Solve one merged group on stream s; per-member statistics into stats.
ebe_status solve_group(ebe_batch* b, Group& g, const double* const* f, double* const* u, const ebe_pcg_opts& o,
                       ebe_pcg_stats* stats, hipStream_t s) {
  const auto t0 = std::chrono::steady_clock::now();
  ebe_mesh* gm = g.mesh;
  const size_t vb = size_t(gm->n_nodes) * 3 * g.nr * sizeof(double);
  EBE_TRY_HIP(launch_fill_zero(g.F.as<void>(), vb, s));
  std::vector<double> host(2 * EBE_MAX_RHS), sc(g.members.size() * EBE_MAX_RHS, 0.0);
  for (size_t k = 0; k < g.members.size(); ++k) {
    const int32_t i = g.members[k];
    const ebe_mesh* m = b->meshes[i];
    const int32_t n = b->nrhs[i];
    EBE_TRY_HIP(launch_case_norms(f[i], nullptr, m->fix.as<uint8_t>(), m->n_nodes, n, g.norms.as<double>(), s));
    EBE_TRY_HIP(hipMemcpyAsync(host.data(), g.norms.as<void>(), n * sizeof(double), hipMemcpyDeviceToHost, s));
    EBE_TRY_HIP(hipStreamSynchronize(s));
    for (int32_t r = 0; r < n; ++r) {
      if (!std::isfinite(host[r])) {
        set_error("mesh %d: NaN or Inf in the right-hand side (case %d)", i, r);
        return EBE_ERR_NONFINITE;
      }
      sc[k * EBE_MAX_RHS + r] = host[r] > 0.0 ? 1.0 / std::sqrt(host[r]) : 0.0;
    }
  }
  EBE_TRY_HIP(hipMemcpyAsync(g.scale.as<void>(), sc.data(), sc.size() * sizeof(double), hipMemcpyHostToDevice, s));
  for (size_t k = 0; k < g.members.size(); ++k) {
    const int32_t i = g.members[k];
    EBE_TRY_HIP(launch_scatter_cases(f[i], g.maps[k]->as<int32_t>(), b->meshes[i]->n_nodes, b->nrhs[i],
                                     g.scale.as<double>() + k * EBE_MAX_RHS, g.F.as<double>(), g.nr, s));
  }
  ebe_pcg_opts og = o;
  og.tol = o.tol / std::sqrt(double(g.members.size()));
  og.use_x0 = 0;
  ebe_pcg_stats gs;
  const ebe_status st = ebe_pcg_solve(gm, g.nr, g.F.as<double>(), g.U.as<double>(), &og, &gs, s);
  if (st < 0) return st;
  for (size_t k = 0; k < g.members.size(); ++k) {
    const int32_t i = g.members[k];
    ebe_mesh* m = b->meshes[i];
    const int32_t n = b->nrhs[i];
    EBE_TRY_HIP(launch_gather_cases(g.U.as<double>(), g.maps[k]->as<int32_t>(), m->n_nodes, n,
                                    g.scale.as<double>() + k * EBE_MAX_RHS, u[i], g.nr, s));
    // the member's own residual, with its own operator
    ebe_status rs = ebe_matvec(m, EBE_F64, n, u[i], g.tmp.as<void>(), 1, s);
    if (rs != EBE_OK) return rs;
    EBE_TRY_HIP(launch_case_norms(f[i], g.tmp.as<double>(), m->fix.as<uint8_t>(), m->n_nodes, n, g.norms.as<double>(), s));
    EBE_TRY_HIP(hipMemcpyAsync(host.data(), g.norms.as<void>(), 2 * n * sizeof(double), hipMemcpyDeviceToHost, s));
    EBE_TRY_HIP(hipStreamSynchronize(s));
    double worst = 0.0;
    for (int32_t r = 0; r < n; ++r)
      if (host[r] > 0.0) worst = std::max(worst, std::sqrt(host[n + r] / host[r]));
    if (stats) {
      ebe_pcg_stats& x = stats[i];
      x = gs;
      x.max_rel_res = worst;
      x.status = st == EBE_OK && worst <= o.tol ? EBE_OK : (st == EBE_OK ? EBE_NOT_CONVERGED : st);
      x.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      x.merged = int32_t(g.members.size());
    }
  }
  return st;
}

}  // namespace

extern "C" {

ebe_status ebe_batch_create(ebe_mesh* const* meshes, int32_t n_mesh, const int32_t* nrhs, ebe_batch** out) {
  if (!out) {
    set_error("ebe_batch_create: out is NULL");
    return EBE_ERR_ARG;
  }
  *out = nullptr;
  if (!meshes || !nrhs || n_mesh < 1) {
    set_error("ebe_batch_create: null argument or n_mesh < 1");
    return EBE_ERR_ARG;
  }
  for (int32_t i = 0; i < n_mesh; ++i) {
    if (!meshes[i] || nrhs[i] < 1 || nrhs[i] > EBE_MAX_RHS) {
      set_error("ebe_batch_create: entry %d has a null mesh or nrhs outside 1..%d", i, EBE_MAX_RHS);
      return EBE_ERR_ARG;
    }
    if (meshes[i]->device != meshes[0]->device) {
      set_error("ebe_batch_create: mesh %d lives on device %d, mesh 0 on device %d", i, meshes[i]->device,
                meshes[0]->device);
      return EBE_ERR_ARG;
    }
    for (int32_t j = 0; j < i; ++j)
      if (meshes[j] == meshes[i]) {
        set_error("ebe_batch_create: mesh %d repeats mesh %d (a handle holds one workspace)", i, j);
        return EBE_ERR_ARG;
      }
  }
  ebe_batch* b = new (std::nothrow) ebe_batch();
  if (!b) {
    set_error("ebe_batch_create: host allocation failed");
    return EBE_ERR_OOM;
  }
  b->meshes.assign(meshes, meshes + n_mesh);
  b->nrhs.assign(nrhs, nrhs + n_mesh);
  b->device = meshes[0]->device;
  int prev = 0;
  hipError_t e = hipGetDevice(&prev);
  if (e == hipSuccess) e = hipSetDevice(b->device);
  const int lanes = std::min<int>(kLanes, n_mesh);
  for (int l = 0; l < lanes && e == hipSuccess; ++l) {
    hipStream_t s = nullptr;
    e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e == hipSuccess) b->lanes.push_back(s);
  }
  (void)hipSetDevice(prev);
  if (e != hipSuccess) {
    set_error("ebe_batch_create: stream creation failed: %s", hipGetErrorString(e));
    ebe_batch_destroy(b);
    return EBE_ERR_HIP;
  }
  *out = b;
  return EBE_OK;
}

ebe_status ebe_batch_set_merge(ebe_batch* b, int64_t max_elems) {
  if (!b || max_elems < 0) {
    set_error("ebe_batch_set_merge: null batch or negative size");
    return EBE_ERR_ARG;
  }
  if (max_elems != b->merge_elems) {
    b->merge_elems = max_elems;
    b->planned = false;
    b->groups.clear();
  }
  return EBE_OK;
}

ebe_status ebe_batch_info(ebe_batch* b, int32_t* n_groups, int32_t* group_of) {
  if (!b) {
    set_error("ebe_batch_info: null batch");
    return EBE_ERR_ARG;
  }
  if (!b->planned) {
    int prev = 0;
    EBE_TRY_HIP(hipGetDevice(&prev));
    EBE_TRY_HIP(hipSetDevice(b->device));
    const ebe_status st = plan(b, b->lanes[0]);
    (void)hipSetDevice(prev);
    if (st != EBE_OK) return st;
  }
  if (n_groups) *n_groups = int32_t(b->groups.size());
  if (group_of) {
    for (size_t i = 0; i < b->meshes.size(); ++i) group_of[i] = -1;
    for (size_t g = 0; g < b->groups.size(); ++g)
      for (int32_t i : b->groups[g]->members) group_of[i] = int32_t(g);
  }
  return EBE_OK;
}

ebe_status ebe_batch_solve(ebe_batch* b, const double* const* f, double* const* u, const ebe_pcg_opts* opts,
                           ebe_pcg_stats* stats, void* stream) {
  if (!b || !f || !u) {
    set_error("ebe_batch_solve: null argument");
    return EBE_ERR_ARG;
  }
  const size_t n = b->meshes.size();
  for (size_t i = 0; i < n; ++i)
    if (!f[i] || !u[i] || !aligned16(f[i]) || !aligned16(u[i])) {
      set_error("ebe_batch_solve: entry %zu has a null or misaligned vector", i);
      return EBE_ERR_ARG;
    }
  ebe_pcg_opts o;
  if (opts) o = *opts;
  else ebe_pcg_default_opts(&o);
  int prev = 0;
  EBE_TRY_HIP(hipGetDevice(&prev));
  EBE_TRY_HIP(hipSetDevice(b->device));
  // The right-hand sides may still be in flight on the caller's stream.
  hipStream_t caller = static_cast<hipStream_t>(stream);
  hipEvent_t ready = nullptr;
  hipError_t e = hipEventCreateWithFlags(&ready, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventRecord(ready, caller);
  for (size_t l = 0; l < b->lanes.size() && e == hipSuccess; ++l) e = hipStreamWaitEvent(b->lanes[l], ready, 0);
  if (e != hipSuccess) {
    if (ready) (void)hipEventDestroy(ready);
    (void)hipSetDevice(prev);
    set_error("ebe_batch_solve: %s", hipGetErrorString(e));
    return EBE_ERR_HIP;
  }
  if (!b->planned) {
    const ebe_status st = plan(b, b->lanes[0]);
    if (st != EBE_OK) {
      (void)hipEventDestroy(ready);
      (void)hipSetDevice(prev);
      return st;
    }
  }
  // jobs: merged groups (index >= 0 into groups) and solo meshes (-1 - mesh), largest first
  // (deterministic solves run every mesh on its own: the merged systems'
  // case scaling sums norms with atomics)
  std::vector<int32_t> jobs;
  std::vector<double> work;
  if (o.deterministic) {
    for (size_t i = 0; i < n; ++i) {
      jobs.push_back(-1 - int32_t(i));
      work.push_back(double(b->meshes[i]->n_elem) * b->nrhs[i]);
    }
  } else {
    for (size_t g = 0; g < b->groups.size(); ++g) {
      jobs.push_back(int32_t(g));
      work.push_back(double(b->groups[g]->mesh->n_elem) * b->groups[g]->nr);
    }
    for (int32_t i : b->solo) {
      jobs.push_back(-1 - i);
      work.push_back(double(b->meshes[i]->n_elem) * b->nrhs[i]);
    }
  }
  std::vector<size_t> order(jobs.size());
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t c) { return work[a] > work[c]; });

  const size_t nj = jobs.size();
  std::vector<ebe_status> status(nj, EBE_ERR_HIP);
  std::vector<std::string> message(nj);
  std::atomic<size_t> next{0};
  auto worker = [&](hipStream_t s) {
    if (hipSetDevice(b->device) != hipSuccess) return;  // every job left unsolved stays EBE_ERR_HIP below
    for (size_t k = next.fetch_add(1); k < nj; k = next.fetch_add(1)) {
      const size_t j = order[k];
      const int32_t id = jobs[j];
      if (id >= 0) {
        status[j] = solve_group(b, *b->groups[id], f, u, o, stats, s);
      } else {
        const int32_t i = -1 - id;
        status[j] = ebe_pcg_solve(b->meshes[i], b->nrhs[i], f[i], u[i], &o, stats ? &stats[i] : nullptr, s);
      }
      if (status[j] < 0) message[j] = ebe_last_error();
    }
  };
  {
    std::vector<std::thread> pool;
    pool.reserve(b->lanes.size());
    try {
      for (hipStream_t s : b->lanes) pool.emplace_back(worker, s);
    } catch (...) {
      // fewer workers than lanes: the ones started still drain the queue
    }
    if (pool.empty()) worker(b->lanes[0]);
    for (auto& t : pool) t.join();
  }
  (void)hipEventDestroy(ready);
  (void)hipSetDevice(prev);

  ebe_status worst = EBE_OK;
  for (size_t j = 0; j < nj; ++j) {
    if (status[j] < 0) {
      const int32_t id = jobs[j];
      if (id >= 0) {
        std::string who;
        for (int32_t i : b->groups[id]->members) who += (who.empty() ? "" : ", ") + std::to_string(i);
        set_error("ebe_batch_solve: merged group %d (meshes %s): %s", id, who.c_str(),
                  message[j].empty() ? ebe_status_string(status[j]) : message[j].c_str());
      } else {
        set_error("ebe_batch_solve: mesh %d: %s", -1 - id,
                  message[j].empty() ? ebe_status_string(status[j]) : message[j].c_str());
      }
      return status[j];
    }
  }
  if (stats)
    for (size_t i = 0; i < n; ++i) worst = std::max(worst, stats[i].status);
  else
    for (size_t j = 0; j < nj; ++j) worst = std::max(worst, status[j]);
  return worst;
}

void ebe_batch_destroy(ebe_batch* b) {
  if (!b) return;
  b->groups.clear();  // merged meshes and their buffers
  for (hipStream_t s : b->lanes) (void)hipStreamDestroy(s);
  delete b;
}

}  // extern "C"
