// Batches of meshes, each with its own set of cases (Section 5 solves its 368
// cases as 23 sets of 16, one set after another).
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstring>
#include <new>
#include <vector>

#include "ebe_internal.h"

using namespace ebe;

struct ebe_batch {
  std::vector<ebe_mesh*> meshes;
  std::vector<int32_t> nrhs;
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
  *out = b;
  return EBE_OK;
}

ebe_status ebe_batch_solve(ebe_batch* b, const double* const* f, double* const* u, const ebe_pcg_opts* opts,
                           ebe_pcg_stats* stats, void* stream) {
  if (!b || !f || !u) {
    set_error("ebe_batch_solve: null argument");
    return EBE_ERR_ARG;
  }
  ebe_status worst = EBE_OK;
  for (size_t i = 0; i < b->meshes.size(); ++i) {
    ebe_status st = ebe_pcg_solve(b->meshes[i], b->nrhs[i], f[i], u[i], opts, stats ? &stats[i] : nullptr, stream);
    if (st < 0) return st;
    if (st > worst) worst = st;
  }
  return worst;
}

void ebe_batch_destroy(ebe_batch* b) { delete b; }

}  // extern "C"
