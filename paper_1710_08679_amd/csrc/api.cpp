// C-ABI entry points of the operators: EBE products, grid transfers, block
// Jacobi and the adjoint element gradient.  Argument checking lives here;
// the kernels assume checked arguments.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ebe_internal.h"

using namespace ebe;

namespace {

ebe_status check_common(const char* fn, const ebe_mesh* m, ebe_dtype dt, int32_t nrhs, const void* x,
                        const void* y) {
  if (!m || !x || !y) {
    set_error("%s: null argument", fn);
    return EBE_ERR_ARG;
  }
  if (dt != EBE_F64 && dt != EBE_F32) {
    set_error("%s: dtype %d is not EBE_F64 or EBE_F32", fn, dt);
    return EBE_ERR_ARG;
  }
  if (nrhs < 1 || nrhs > EBE_MAX_RHS) {
    set_error("%s: nrhs %d outside 1..%d", fn, nrhs, EBE_MAX_RHS);
    return EBE_ERR_ARG;
  }
  if (x == y) {
    set_error("%s: input and output must not alias", fn);
    return EBE_ERR_ARG;
  }
  if (!aligned16(x) || !aligned16(y)) {
    set_error("%s: device buffers must be 16-byte aligned", fn);
    return EBE_ERR_ARG;
  }
  return EBE_OK;
}

ebe_status hip_status(const char* fn, hipError_t e) {
  if (e == hipSuccess) return EBE_OK;
  set_error("%s: %s", fn, hipGetErrorString(e));
  return EBE_ERR_HIP;
}

}  // namespace

namespace ebe {

ebe_status ensure_geometry(ebe_mesh* m, ebe_dtype dt, hipStream_t s) {
  const int k = dt == EBE_F64 ? 0 : 1;
  if (m->geo_ready[k]) return EBE_OK;
  ebe_status st = m->geo[k].alloc(size_t(m->n_elem) * 16 * (dt == EBE_F64 ? 8 : 4));
  if (st != EBE_OK) return st;
  EBE_TRY_HIP(launch_geometry(m, dt, m->geo[k].as<void>(), s));
  m->geo_ready[k] = true;
  return EBE_OK;
}

ebe_status ensure_assembled(ebe_mesh* m, ebe_dtype dt, hipStream_t s) {
  const int k = dt == EBE_F64 ? 0 : 1;
  if (m->k1.ready[k]) return EBE_OK;
  const size_t n = size_t(m->k1.slots) * 9 * kSliceRows;
  ebe_status st = m->k1.val[0].alloc(n * sizeof(double));  // FP64 values are formed first in any case
  if (st == EBE_OK && k == 1) st = m->k1.val[1].alloc(n * sizeof(float));
  if (st != EBE_OK) return st;
  EBE_TRY_HIP(launch_assemble_p1(m, !m->k1.ready[0], k == 1, s));
  m->k1.ready[0] = true;
  m->k1.ready[k] = true;
  return EBE_OK;
}

ebe_status ensure_level2(ebe_mesh* m, ebe_dtype dt, hipStream_t s) {
  const int k = dt == EBE_F64 ? 0 : 1;
  if (m->a2.ready[k]) return EBE_OK;
  if (m->a2_maxlen > kA2MaxRow) {
    set_error("level 2: a coarse row couples %d aggregates (at most %d); use MG2", m->a2_maxlen, kA2MaxRow);
    return EBE_ERR_ARG;
  }
  // P2 and A2 are formed from the FP64 K1 blocks and the level-1 block Jacobi
  ebe_status st = ensure_assembled(m, EBE_F64, s);
  if (st == EBE_OK) st = ensure_blocks(m, s);
  const size_t n = std::max<size_t>(size_t(m->a2.slots) * 9 * kSliceRows, 1);
  const size_t np = std::max<size_t>(size_t(m->n_vertices) * m->p2_width * 9, 1);
  if (st == EBE_OK) st = m->a2.val[0].alloc(n * sizeof(double));
  if (st == EBE_OK && k == 1) st = m->a2.val[1].alloc(n * sizeof(float));
  if (st == EBE_OK) st = m->p2_val[0].alloc(np * sizeof(double));
  if (st == EBE_OK) st = m->p2_val[1].alloc(np * sizeof(float));
  if (st != EBE_OK) return st;
  const bool fresh = !m->a2.ready[0];
  EBE_TRY_HIP(launch_assemble_a2(m, fresh, k == 1, s));
  if (fresh) {  // the level-2 block Jacobi goes with the FP64 values
    const size_t na = size_t(std::max<int64_t>(m->n_agg, 1));
    DBuf tmp;
    st = tmp.alloc(na * 6 * sizeof(double));
    if (st == EBE_OK) st = m->minv64[2].alloc(na * 6 * sizeof(double));
    if (st == EBE_OK) st = m->minv32[2].alloc(na * 6 * sizeof(float));
    if (st != EBE_OK) return st;
    EBE_TRY_HIP(launch_asm_diag(m->a2, tmp.as<double>(), s));
    EBE_TRY_HIP(launch_invert_blocks(m, 2, tmp.as<double>(), m->minv64[2].as<double>(), m->minv32[2].as<float>(),
                                     s));
    EBE_TRY_HIP(hipStreamSynchronize(s));  // tmp is freed at scope exit
  }
  m->a2.ready[0] = true;
  m->a2.ready[k] = true;
  return EBE_OK;
}

ebe_status ensure_half(ebe_mesh* m, int level, hipStream_t s) {
  AsmOp& op = level == 2 ? m->a2 : m->k1;
  if (op.ready16) return EBE_OK;
  ebe_status st = level == 2 ? ensure_level2(m, EBE_F64, s) : ensure_assembled(m, EBE_F64, s);
  if (st != EBE_OK) return st;
  const int64_t n = op.slots * 9 * kSliceRows;
  DBuf mx;
  if ((st = op.val16.alloc(std::max<size_t>(size_t(n) * 2, 2))) != EBE_OK) return st;
  if ((st = mx.alloc(sizeof(unsigned long long))) != EBE_OK) return st;
  EBE_TRY_HIP(launch_absmax(op.val[0].as<double>(), n, mx.as<unsigned long long>(), s));
  unsigned long long bits = 0;
  EBE_TRY_HIP(hipMemcpyAsync(&bits, mx.as<void>(), sizeof(bits), hipMemcpyDeviceToHost, s));
  EBE_TRY_HIP(hipStreamSynchronize(s));
  double amax = 0.0;
  std::memcpy(&amax, &bits, sizeof(amax));
  // values scaled so the largest is 2^14: inside FP16's range with room, small
  // entries keep FP16's 11-bit significand down to 2^-14 of the largest
  op.half_scale = amax > 0.0 ? amax / 16384.0 : 1.0;
  EBE_TRY_HIP(launch_to_f16(op.val[0].as<double>(), op.val16.as<void>(), n, 1.0 / op.half_scale, s));
  EBE_TRY_HIP(hipStreamSynchronize(s));
  op.ready16 = true;
  return EBE_OK;
}

ebe_status prepare_products(ebe_mesh* m, int level, ebe_dtype dt, int nrhs, hipStream_t s) {
  ebe_status st = ensure_stage(m, nrhs, dt == EBE_F64 ? 8 : 4);
  if (st == EBE_OK) st = ensure_geometry(m, dt, s);
  if (st == EBE_OK && level == 1 && product_form(m, 1, dt, nrhs) == EBE_FORM_ASSEMBLED)
    st = ensure_assembled(m, dt, s);
  return st;
}

// Form and invert the 3x3 block-Jacobi blocks of both levels (once per material).
ebe_status ensure_blocks(ebe_mesh* m, hipStream_t s) {
  if (m->minv_ready) return EBE_OK;
  DBuf tmp;
  ebe_status st = tmp.alloc(size_t(m->n_nodes) * 6 * sizeof(double));
  if (st != EBE_OK) return st;
  for (int level = 0; level < 2; ++level) {
    const int64_t n = level == 0 ? m->n_nodes : m->n_vertices;
    if ((st = m->minv64[level].alloc(size_t(n) * 6 * sizeof(double))) != EBE_OK) return st;
    if ((st = m->minv32[level].alloc(size_t(n) * 6 * sizeof(float))) != EBE_OK) return st;
    EBE_TRY_HIP(launch_diag_blocks(m, level, tmp.as<double>(), s));
    EBE_TRY_HIP(launch_invert_blocks(m, level, tmp.as<double>(), m->minv64[level].as<double>(),
                                     m->minv32[level].as<float>(), s));
  }
  // tmp is freed at scope exit; make sure the kernels that read it are done
  EBE_TRY_HIP(hipStreamSynchronize(s));
  m->minv_ready = true;
  return EBE_OK;
}

}  // namespace ebe

extern "C" {

ebe_status ebe_matvec(ebe_mesh* m, ebe_dtype dt, int32_t nrhs, const void* x, void* y, int32_t apply_bc,
                      void* stream) {
  ebe_status st = check_common("ebe_matvec", m, dt, nrhs, x, y);
  if (st != EBE_OK) return st;
  if ((st = prepare_products(m, 0, dt, nrhs, static_cast<hipStream_t>(stream))) != EBE_OK) return st;
  return hip_status("ebe_matvec", launch_ebe_p2(m, dt, nrhs, x, y, apply_bc && m->has_bc,
                                                static_cast<hipStream_t>(stream)));
}

ebe_status ebe_matvec_noalloc(ebe_mesh* m, ebe_dtype dt, int32_t nrhs, const void* x, void* y, int32_t apply_bc,
                              void* stream) {
  ebe_status st = check_common("ebe_matvec_noalloc", m, dt, nrhs, x, y);
  if (st != EBE_OK) return st;
  const size_t need = size_t(m->pl[0].nslots) * 3 * size_t(nrhs) * (dt == EBE_F64 ? 8 : 4);
  if (need > kNoAllocScratchBytes) {
    set_error("ebe_matvec_noalloc: this mesh stages %zu bytes of shared-node sums at nrhs %d; the "
              "allocation-free scratch holds %zu (use ebe_matvec, or fewer cases per call)",
              need, nrhs, kNoAllocScratchBytes);
    return EBE_ERR_ARG;
  }
  void* stage = nullptr;
  if ((st = noalloc_scratch(m->device, &stage)) != EBE_OK) return st;
  return hip_status("ebe_matvec_noalloc", launch_ebe_noalloc(m, dt, nrhs, x, y, apply_bc && m->has_bc, stage,
                                                             static_cast<hipStream_t>(stream)));
}

ebe_status ebe_matvec_add(ebe_mesh* m, ebe_dtype dt, int32_t nrhs, const void* x, void* y, int32_t apply_bc,
                          void* stream) {
  ebe_status st = check_common("ebe_matvec_add", m, dt, nrhs, x, y);
  if (st != EBE_OK) return st;
  if ((st = prepare_products(m, 0, dt, nrhs, static_cast<hipStream_t>(stream))) != EBE_OK) return st;
  const bool bc = apply_bc && m->has_bc;
  return hip_status("ebe_matvec_add",
                    launch_ebe(m, 2, dt, nrhs, x, y, bc, bc, true, nullptr, static_cast<hipStream_t>(stream)));
}

ebe_status ebe_matvec_p1(ebe_mesh* m, ebe_dtype dt, int32_t nrhs, const void* x, void* y, int32_t apply_bc,
                         void* stream) {
  ebe_status st = check_common("ebe_matvec_p1", m, dt, nrhs, x, y);
  if (st != EBE_OK) return st;
  if ((st = prepare_products(m, 1, dt, nrhs, static_cast<hipStream_t>(stream))) != EBE_OK) return st;
  return hip_status("ebe_matvec_p1", launch_ebe_p1(m, dt, nrhs, x, y, apply_bc && m->has_bc,
                                                   static_cast<hipStream_t>(stream)));
}

ebe_status ebe_prolong_p1(ebe_mesh* m, ebe_dtype dt, int32_t nrhs, const void* x, void* y, int32_t apply_bc,
                          void* stream) {
  ebe_status st = check_common("ebe_prolong_p1", m, dt, nrhs, x, y);
  if (st != EBE_OK) return st;
  return hip_status("ebe_prolong_p1", launch_prolong(m, dt, nrhs, x, y, apply_bc && m->has_bc,
                                                     static_cast<hipStream_t>(stream)));
}

ebe_status ebe_restrict_p1(ebe_mesh* m, ebe_dtype dt, int32_t nrhs, const void* x, void* y, int32_t apply_bc,
                           void* stream) {
  ebe_status st = check_common("ebe_restrict_p1", m, dt, nrhs, x, y);
  if (st != EBE_OK) return st;
  return hip_status("ebe_restrict_p1", launch_restrict(m, dt, nrhs, x, y, apply_bc && m->has_bc,
                                                       static_cast<hipStream_t>(stream)));
}

ebe_status ebe_patch_info(const ebe_mesh* m, int32_t level, int64_t* n_patches, int64_t* n_shared,
                          int64_t* n_staged, int32_t* n_colours) {
  if (!m || (level != 0 && level != 1)) {
    set_error("ebe_patch_info: null mesh or level not 0/1");
    return EBE_ERR_ARG;
  }
  const PatchLevel& L = m->pl[level];
  if (n_patches) *n_patches = L.npatch;
  if (n_shared) *n_shared = L.nshared;
  if (n_staged) *n_staged = L.nslots;
  if (n_colours) *n_colours = L.coff.empty() ? 0 : int32_t(L.coff.size() - 1);
  return EBE_OK;
}

ebe_status ebe_level2_info(const ebe_mesh* m, int64_t* n_agg, int32_t* agg_host) {
  if (!m) {
    set_error("ebe_level2_info: null mesh");
    return EBE_ERR_ARG;
  }
  if (n_agg) *n_agg = m->n_agg;
  if (agg_host)
    EBE_TRY_HIP(hipMemcpy(agg_host, m->agg.as<void>(), size_t(m->n_vertices) * sizeof(int32_t),
                          hipMemcpyDeviceToHost));
  return EBE_OK;
}

ebe_status ebe_matvec_l2(ebe_mesh* m, ebe_dtype dt, int32_t nrhs, const void* x, void* y, int32_t apply_bc,
                         void* stream) {
  ebe_status st = check_common("ebe_matvec_l2", m, dt, nrhs, x, y);
  if (st != EBE_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if ((st = ensure_level2(m, dt, s)) != EBE_OK) return st;
  const bool bc = apply_bc != 0;
  return hip_status("ebe_matvec_l2", launch_level2(m, dt, nrhs, x, y, bc, bc, false, nullptr, s));
}

ebe_status ebe_prolong_l2(ebe_mesh* m, ebe_dtype dt, int32_t nrhs, const void* x, void* y, void* stream) {
  ebe_status st = check_common("ebe_prolong_l2", m, dt, nrhs, x, y);
  if (st != EBE_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if ((st = ensure_level2(m, EBE_F64, s)) != EBE_OK) return st;  // P2 is formed with A2
  return hip_status("ebe_prolong_l2", launch_prolong_p2(m, dt, nrhs, x, y, s));
}

ebe_status ebe_restrict_l2(ebe_mesh* m, ebe_dtype dt, int32_t nrhs, const void* x, void* y, void* stream) {
  ebe_status st = check_common("ebe_restrict_l2", m, dt, nrhs, x, y);
  if (st != EBE_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if ((st = ensure_level2(m, EBE_F64, s)) != EBE_OK) return st;  // P2 is formed with A2
  return hip_status("ebe_restrict_l2", launch_restrict_p2(m, dt, nrhs, x, y, s));
}

ebe_status ebe_diag_blocks(ebe_mesh* m, int32_t level, double* blocks, void* stream) {
  if (!m || !blocks || level < 0 || level > 2) {
    set_error("ebe_diag_blocks: null argument or level not 0/1/2");
    return EBE_ERR_ARG;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t n = level_rows(m, level);
  DBuf tmp;
  ebe_status st = tmp.alloc(size_t(std::max<int64_t>(n, 1)) * 6 * sizeof(double));
  if (st != EBE_OK) return st;
  if (level == 2) {
    if ((st = ensure_level2(m, EBE_F64, s)) != EBE_OK) return st;
    EBE_TRY_HIP(launch_asm_diag(m->a2, tmp.as<double>(), s));
  } else {
    EBE_TRY_HIP(launch_diag_blocks(m, level, tmp.as<double>(), s));
  }
  EBE_TRY_HIP(launch_expand_blocks(n, tmp.as<double>(), blocks, s));
  EBE_TRY_HIP(hipStreamSynchronize(s));
  return EBE_OK;
}

ebe_status ebe_block_jacobi(ebe_mesh* m, int32_t level, ebe_dtype dt, int32_t nrhs, const void* x, void* y,
                            void* stream) {
  ebe_status st = check_common("ebe_block_jacobi", m, dt, nrhs, x, y);
  if (st != EBE_OK) return st;
  if (level < 0 || level > 2) {
    set_error("ebe_block_jacobi: level %d not 0/1/2", level);
    return EBE_ERR_ARG;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  if ((st = ensure_blocks(m, s)) != EBE_OK) return st;
  if (level == 2 && (st = ensure_level2(m, EBE_F64, s)) != EBE_OK) return st;
  return hip_status("ebe_block_jacobi", launch_bjacobi(m, level, dt, nrhs, x, y, s));
}

ebe_status ebe_adjoint_grad(ebe_mesh* m, ebe_dtype dt, int32_t nrhs, const void* u, const void* lam, void* g,
                            void* stream) {
  ebe_status st = check_common("ebe_adjoint_grad", m, dt, nrhs, u, g);
  if (st == EBE_OK && m->curved) {
    set_error("ebe_adjoint_grad: not supported on a mesh of curved elements");
    return EBE_ERR_ARG;
  }
  if (st != EBE_OK) return st;
  if (!lam || lam == g || !aligned16(lam)) {
    set_error("ebe_adjoint_grad: lam is NULL, aliases g or is not 16-byte aligned");
    return EBE_ERR_ARG;
  }
  return hip_status("ebe_adjoint_grad", launch_adjoint(m, dt, nrhs, u, lam, g, static_cast<hipStream_t>(stream)));
}

}  // extern "C"
