// Per-mesh choice of the EBE product form.  Which form of the patch kernel
// is faster depends on the dtype, the number of cases and the mesh (patch
// node counts, how many nodes are shared), so it is measured: all forms run
// the same product a few times on the mesh itself and the faster is kept for
// that (level, dtype, nrhs).  Search over implementation parameters, as the
// paper does for its own kernels (Section 4), only automated.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>

#include "ebe_internal.h"

using namespace ebe;

namespace {

constexpr int kRuns = 3;

bool valid_args(const ebe_mesh* m, int32_t level, ebe_dtype dt, int32_t nrhs, const char* fn) {
  if (!m || (level != 0 && level != 1) || (dt != EBE_F64 && dt != EBE_F32) || nrhs < 1 || nrhs > EBE_MAX_RHS) {
    set_error("%s: null mesh, level not 0/1, bad dtype or nrhs outside 1..%d", fn, EBE_MAX_RHS);
    return false;
  }
  return true;
}

}  // namespace

namespace ebe {

ebe_status tune_product(ebe_mesh* m, int level, ebe_dtype dt, int nrhs, const void* x, void* y, hipStream_t s,
                        double ms[EBE_NUM_FORMS]) {
  const int order = level == 0 ? 2 : 1;
  ebe_status st = ensure_stage(m, nrhs, dt == EBE_F64 ? 8 : 4);
  if (st == EBE_OK) st = ensure_geometry(m, dt, s);
  if (st == EBE_OK && level == 1) st = ensure_assembled(m, dt, s);
  if (st != EBE_OK) return st;
  hipEvent_t a = nullptr, b = nullptr;
  EBE_TRY_HIP(hipEventCreate(&a));
  hipError_t e = hipEventCreate(&b);
  const int lv = level, k = dt == EBE_F64 ? 0 : 1;
  double best[EBE_NUM_FORMS];
  int best_var[EBE_NUM_FORMS] = {};
  for (int f = 0; f < EBE_NUM_FORMS; ++f) best[f] = DBL_MAX;
  for (int form = 0; form < EBE_NUM_FORMS && e == hipSuccess; ++form) {
    if (!form_usable(m, order, form, dt, nrhs)) continue;
    // the patch kernels come in two variants: pipelined and coloured with
    // the element geometry kept in LDS or read per work-item, gather and
    // staged with the geometry read from the cache or formed from the corner
    // coordinates, deterministic with staging or colour by colour; the
    // assembled form comes in three tiles: measure them all
    const bool curved = order == 2 && m->curved;
    const int nvar = form == EBE_FORM_ASSEMBLED ? 3  // tiles: cases per work-item, slots per trip
                     : (form == EBE_FORM_PIPELINED || form == EBE_FORM_COLOURED ||
                        ((form == EBE_FORM_GATHER || form == EBE_FORM_STAGED) && !curved) ||
                        (form == EBE_FORM_DETERMINISTIC && m->pl[0].coff.size() > 1))
                         ? 2
                         : 1;
    for (int var = 0; var < nvar && e == hipSuccess; ++var) {
      m->fvar[lv][k][nrhs] = int8_t(var);
      e = launch_ebe_form(m, order, form, dt, nrhs, x, y, false, m->has_bc, false, nullptr, s);  // warm-up
      for (int r = 0; r < kRuns && e == hipSuccess; ++r) {
        e = hipEventRecord(a, s);
        if (e == hipSuccess) e = launch_ebe_form(m, order, form, dt, nrhs, x, y, false, m->has_bc, false, nullptr, s);
        if (e == hipSuccess) e = hipEventRecord(b, s);
        if (e == hipSuccess) e = hipEventSynchronize(b);
        float t = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
        if (e == hipSuccess && double(t) < best[form]) {
          best[form] = double(t);
          best_var[form] = var;
        }
      }
    }
  }
  (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  if (e != hipSuccess) {
    m->fvar[lv][k][nrhs] = 0;
    set_error("autotune: %s", hipGetErrorString(e));
    return EBE_ERR_HIP;
  }
  int pick = 0;
  for (int f = 1; f < EBE_NUM_FORMS; ++f)
    if (best[f] < best[pick]) pick = f;
  m->form[lv][k][nrhs] = int8_t(pick);
  m->fvar[lv][k][nrhs] = int8_t(best_var[pick]);
  if (ms)
    for (int f = 0; f < EBE_NUM_FORMS; ++f) ms[f] = form_usable(m, order, f, dt, nrhs) ? best[f] : -1.0;
  return EBE_OK;
}

}  // namespace ebe

extern "C" {

ebe_status ebe_autotune(ebe_mesh* m, int32_t level, ebe_dtype dt, int32_t nrhs, void* stream, double* ms_out) {
  if (!valid_args(m, level, dt, nrhs, "ebe_autotune")) return EBE_ERR_ARG;
  const int64_t rows = level == 0 ? m->n_nodes : m->n_vertices;
  const size_t bytes = size_t(rows) * 3 * size_t(nrhs) * (dt == EBE_F64 ? 8 : 4);
  DBuf x, y;
  ebe_status st = x.alloc(bytes);
  if (st == EBE_OK) st = y.alloc(bytes);
  if (st != EBE_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  EBE_TRY_HIP(launch_fill_zero(x.as<void>(), bytes, s));
  double ms[EBE_NUM_FORMS];
  st = tune_product(m, level, dt, nrhs, x.as<void>(), y.as<void>(), s, ms);
  if (st == EBE_OK && ms_out)
    for (int f = 0; f < EBE_NUM_FORMS; ++f) ms_out[f] = ms[f];
  EBE_TRY_HIP(hipStreamSynchronize(s));  // the temporaries are freed on return
  return st;
}

ebe_status ebe_set_product_form(ebe_mesh* m, int32_t level, ebe_dtype dt, int32_t nrhs, int32_t form) {
  if (!valid_args(m, level, dt, nrhs, "ebe_set_product_form")) return EBE_ERR_ARG;
  if (form != EBE_FORM_AUTO && !form_available(level == 0 ? 2 : 1, form)) {
    set_error("ebe_set_product_form: form %d is not EBE_FORM_AUTO or a form of level %d", form, level);
    return EBE_ERR_ARG;
  }
  m->form[level][dt == EBE_F64 ? 0 : 1][nrhs] = int8_t(form);
  m->fvar[level][dt == EBE_F64 ? 0 : 1][nrhs] = 0;
  return EBE_OK;
}

ebe_status ebe_set_product_variant(ebe_mesh* m, int32_t level, ebe_dtype dt, int32_t nrhs, int32_t variant) {
  if (!valid_args(m, level, dt, nrhs, "ebe_set_product_variant")) return EBE_ERR_ARG;
  if (variant < 0 || variant > 2) {
    set_error("ebe_set_product_variant: variant %d is not 0, 1 or 2", variant);
    return EBE_ERR_ARG;
  }
  m->fvar[level][dt == EBE_F64 ? 0 : 1][nrhs] = int8_t(variant);
  return EBE_OK;
}

ebe_status ebe_get_product_variant(const ebe_mesh* m, int32_t level, ebe_dtype dt, int32_t nrhs, int32_t* variant) {
  if (!valid_args(m, level, dt, nrhs, "ebe_get_product_variant") || !variant) {
    if (m && !variant) set_error("ebe_get_product_variant: variant is NULL");
    return EBE_ERR_ARG;
  }
  *variant = m->fvar[level][dt == EBE_F64 ? 0 : 1][nrhs];
  return EBE_OK;
}

ebe_status ebe_get_product_form(const ebe_mesh* m, int32_t level, ebe_dtype dt, int32_t nrhs, int32_t* form) {
  if (!valid_args(m, level, dt, nrhs, "ebe_get_product_form") || !form) {
    if (m && !form) set_error("ebe_get_product_form: form is NULL");
    return EBE_ERR_ARG;
  }
  *form = product_form(m, level == 0 ? 2 : 1, dt, nrhs);
  return EBE_OK;
}

}  // extern "C"
