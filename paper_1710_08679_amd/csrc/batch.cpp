// Batches of meshes, each with its own set of cases.  Section 5 solves its
// 368 cases as 23 sets of 16, one set after another; a batch instead keeps
// several solves in flight at once so that meshes too small to fill the GPU
// share it.
//
// Each of up to kLanes worker threads owns a stream (default priority) and
// takes the next unsolved mesh, largest first (element count x nrhs), and
// runs the ordinary solver on it.  The solver synchronises only its own
// stream, so the kernels of different meshes overlap on the GPU's hardware
// queues while each worker waits at its convergence checks.  A mesh handle
// holds one workspace, so a mesh appears at most once in a batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "ebe_internal.h"

using namespace ebe;

namespace {
constexpr int kLanes = 4;  // concurrent solves: one per hardware queue a process gets by default
}

struct ebe_batch {
  std::vector<ebe_mesh*> meshes;
  std::vector<int32_t> nrhs;
  std::vector<int32_t> order;       // mesh indices, largest solve first
  std::vector<hipStream_t> lanes;   // worker streams
  int device = 0;
};

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
  b->order.resize(n_mesh);
  std::iota(b->order.begin(), b->order.end(), 0);
  std::stable_sort(b->order.begin(), b->order.end(), [&](int32_t a, int32_t c) {
    return double(b->meshes[a]->n_elem) * b->nrhs[a] > double(b->meshes[c]->n_elem) * b->nrhs[c];
  });
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

ebe_status ebe_batch_solve(ebe_batch* b, const double* const* f, double* const* u, const ebe_pcg_opts* opts,
                           ebe_pcg_stats* stats, void* stream) {
  if (!b || !f || !u) {
    set_error("ebe_batch_solve: null argument");
    return EBE_ERR_ARG;
  }
  const size_t n = b->meshes.size();
  for (size_t i = 0; i < n; ++i)
    if (!f[i] || !u[i]) {
      set_error("ebe_batch_solve: entry %zu has a null vector", i);
      return EBE_ERR_ARG;
    }
  // The right-hand sides may still be in flight on the caller's stream.
  hipStream_t caller = static_cast<hipStream_t>(stream);
  hipEvent_t ready = nullptr;
  int prev = 0;
  EBE_TRY_HIP(hipGetDevice(&prev));
  EBE_TRY_HIP(hipSetDevice(b->device));
  hipError_t e = hipEventCreateWithFlags(&ready, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventRecord(ready, caller);
  for (size_t l = 0; l < b->lanes.size() && e == hipSuccess; ++l) e = hipStreamWaitEvent(b->lanes[l], ready, 0);
  if (e != hipSuccess) {
    if (ready) (void)hipEventDestroy(ready);
    (void)hipSetDevice(prev);
    set_error("ebe_batch_solve: %s", hipGetErrorString(e));
    return EBE_ERR_HIP;
  }

  std::vector<ebe_status> status(n, EBE_OK);
  std::vector<std::string> message(n);
  std::atomic<size_t> next{0};
  auto worker = [&](hipStream_t s) {
    if (hipSetDevice(b->device) != hipSuccess) return;  // every mesh left unsolved stays EBE_ERR_HIP below
    for (size_t k = next.fetch_add(1); k < n; k = next.fetch_add(1)) {
      const int32_t i = b->order[k];
      status[i] = ebe_pcg_solve(b->meshes[i], b->nrhs[i], f[i], u[i], opts, stats ? &stats[i] : nullptr, s);
      if (status[i] < 0) message[i] = ebe_last_error();
    }
  };
  std::fill(status.begin(), status.end(), EBE_ERR_HIP);
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
  for (size_t i = 0; i < n; ++i) {
    if (status[i] < 0) {
      set_error("ebe_batch_solve: mesh %zu: %s", i,
                message[i].empty() ? ebe_status_string(status[i]) : message[i].c_str());
      return status[i];
    }
    worst = std::max(worst, status[i]);
  }
  return worst;
}

void ebe_batch_destroy(ebe_batch* b) {
  if (!b) return;
  for (hipStream_t s : b->lanes) (void)hipStreamDestroy(s);
  delete b;
}

}  // extern "C"
