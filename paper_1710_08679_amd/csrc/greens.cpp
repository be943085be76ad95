// C-ABI entry points of the Green's-function pipeline (Section 5, Eq. (4) and
// Eq. (5); split-node fault loading, Section 2): the fault handle, the
// split-node forces of unit-slip basis functions, the Green's functions at
// observation points computed in sets of at most 16 basis functions (one
// multi-case solve per set, as the application solves its cases in sets of
// 16), and the regularised least-squares inversion over a set of weights with
// the L-curve corner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

#include "greens.h"

using namespace ebe;

extern "C" {

ebe_status ebe_fault_create(ebe_mesh* m, const int8_t* sides, int64_t n_fault_nodes, const int32_t* fault_nodes,
                            int32_t n_basis, const double* basis, const double* dirs, ebe_fault** out) {
  if (!out) {
    set_error("ebe_fault_create: out is NULL");
    return EBE_ERR_ARG;
  }
  *out = nullptr;
  if (!m || !sides || n_fault_nodes < 1 || !fault_nodes || n_basis < 1 || !basis || !dirs) {
    set_error("ebe_fault_create: null argument, no fault node or no basis function");
    return EBE_ERR_ARG;
  }
  if (m->curved) {
    set_error("ebe_fault_create: not supported on a mesh of curved elements");
    return EBE_ERR_ARG;
  }
  const int64_t N = m->n_nodes, E = m->n_elem;
  std::vector<int32_t> row(N, -1);
  for (int64_t i = 0; i < n_fault_nodes; ++i) {
    const int32_t v = fault_nodes[i];
    if (v < 0 || v >= N || row[v] >= 0) {
      set_error("ebe_fault_create: fault node %lld (id %d) out of range or repeated", (long long)i, v);
      return EBE_ERR_INDEX;
    }
    row[v] = int32_t(i);
  }
  for (int64_t i = 0; i < n_fault_nodes * n_basis; ++i)
    if (!std::isfinite(basis[i])) {
      set_error("ebe_fault_create: non-finite basis value at %lld", (long long)i);
      return EBE_ERR_NONFINITE;
    }
  for (int32_t i = 0; i < 3 * n_basis; ++i)
    if (!std::isfinite(dirs[i])) {
      set_error("ebe_fault_create: non-finite slip direction at %d", i);
      return EBE_ERR_NONFINITE;
    }
  // the element's nodes, from the device connectivity (fix bits masked off)
  std::vector<int32_t> conn(size_t(E) * 10);
  EBE_TRY_HIP(hipMemcpy(conn.data(), m->conn.as<void>(), conn.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
  std::vector<int32_t> fel, frow;
  std::vector<int8_t> fside;
  for (int64_t e = 0; e < E; ++e) {
    if (sides[e] != 0 && sides[e] != 1 && sides[e] != -1) {
      set_error("ebe_fault_create: side of element %lld is %d (not -1, 0, 1)", (long long)e, int(sides[e]));
      return EBE_ERR_ARG;
    }
    bool touch = false;
    for (int a = 0; a < 10; ++a) touch |= row[conn[size_t(e) * 10 + a] & kIdxMask] >= 0;
    if (touch && sides[e] == 0) {
      set_error("ebe_fault_create: element %lld touches a fault node but has side 0", (long long)e);
      return EBE_ERR_ARG;
    }
    if (sides[e] == 0) continue;
    fel.push_back(int32_t(e));
    fside.push_back(sides[e]);
    for (int a = 0; a < 10; ++a) frow.push_back(row[conn[size_t(e) * 10 + a] & kIdxMask]);
  }
  ebe_fault* fl = new (std::nothrow) ebe_fault();
  if (!fl) {
    set_error("ebe_fault_create: host allocation failed");
    return EBE_ERR_OOM;
  }
  fl->mesh = m;
  fl->nbasis = n_basis;
  fl->nfault = n_fault_nodes;
  fl->nfel = int32_t(fel.size());
  auto up = [&](DBuf& b, const void* h, size_t bytes) -> ebe_status {
    ebe_status st = b.alloc(std::max<size_t>(bytes, 1));
    if (st != EBE_OK) return st;
    if (bytes) EBE_TRY_HIP(hipMemcpy(b.as<void>(), h, bytes, hipMemcpyHostToDevice));
    return EBE_OK;
  };
  ebe_status st = up(fl->fel, fel.data(), fel.size() * sizeof(int32_t));
  if (st == EBE_OK) st = up(fl->fside, fside.data(), fside.size());
  if (st == EBE_OK) st = up(fl->frow, frow.data(), frow.size() * sizeof(int32_t));
  if (st == EBE_OK) st = up(fl->basis, basis, size_t(n_fault_nodes) * n_basis * sizeof(double));
  if (st == EBE_OK) st = up(fl->dirs, dirs, size_t(n_basis) * 3 * sizeof(double));
  if (st != EBE_OK) {
    delete fl;
    return st;
  }
  *out = fl;
  return EBE_OK;
}

void ebe_fault_destroy(ebe_fault* fl) { delete fl; }

ebe_status ebe_split_node_forces(ebe_fault* fl, int32_t col0, int32_t nrhs, double* f, void* stream) {
  if (!fl || !f || nrhs < 1 || nrhs > EBE_MAX_RHS || col0 < 0 || col0 + nrhs > fl->nbasis) {
    set_error("ebe_split_node_forces: null argument, nrhs outside 1..%d or columns outside 0..%d", EBE_MAX_RHS,
              fl ? fl->nbasis - 1 : 0);
    return EBE_ERR_ARG;
  }
  if (!aligned16(f)) {
    set_error("ebe_split_node_forces: f must be 16-byte aligned");
    return EBE_ERR_ARG;
  }
  const hipError_t e = launch_split_forces(fl->mesh, fl->fel.as<int32_t>(), fl->fside.as<int8_t>(),
                                           fl->frow.as<int32_t>(), fl->basis.as<double>(), fl->dirs.as<double>(),
                                           fl->nbasis, fl->nfel, col0, nrhs, f, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) {
    set_error("ebe_split_node_forces: %s", hipGetErrorString(e));
    return EBE_ERR_HIP;
  }
  return EBE_OK;
}

ebe_status ebe_greens_functions(ebe_fault* fl, int32_t n_stations, const int32_t* stations_host, double* G,
                                const ebe_pcg_opts* opts, ebe_pcg_stats* stats, void* stream) {
  if (!fl || n_stations < 1 || !stations_host || !G) {
    set_error("ebe_greens_functions: null argument or no station");
    return EBE_ERR_ARG;
  }
  ebe_mesh* m = fl->mesh;
  for (int32_t i = 0; i < n_stations; ++i)
    if (stations_host[i] < 0 || stations_host[i] >= m->n_nodes) {
      set_error("ebe_greens_functions: station %d is node %d, outside 0..%lld", i, stations_host[i],
                (long long)m->n_nodes - 1);
      return EBE_ERR_INDEX;
    }
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t vbytes = size_t(m->n_nodes) * 3 * EBE_MAX_RHS * sizeof(double);
  DBuf stations;
  ebe_status st = fl->f.alloc(vbytes);
  if (st == EBE_OK) st = fl->u.alloc(vbytes);
  if (st == EBE_OK) st = stations.alloc(size_t(n_stations) * sizeof(int32_t));
  if (st != EBE_OK) return st;
  EBE_TRY_HIP(hipMemcpyAsync(stations.as<void>(), stations_host, size_t(n_stations) * sizeof(int32_t),
                             hipMemcpyHostToDevice, s));
  ebe_status worst = EBE_OK;
  for (int32_t c0 = 0, set = 0; c0 < fl->nbasis; c0 += EBE_MAX_RHS, ++set) {
    const int32_t nr = std::min<int32_t>(EBE_MAX_RHS, fl->nbasis - c0);
    if ((st = ebe_split_node_forces(fl, c0, nr, fl->f.as<double>(), stream)) != EBE_OK) return st;
    st = ebe_pcg_solve(m, nr, fl->f.as<double>(), fl->u.as<double>(), opts, stats ? &stats[set] : nullptr, stream);
    if (st < 0) return st;
    worst = std::max(worst, st);
    const hipError_t e =
        launch_gather_obs(fl->u.as<double>(), nr, stations.as<int32_t>(), n_stations, G, fl->nbasis, c0, s);
    if (e != hipSuccess) {
      set_error("ebe_greens_functions: %s", hipGetErrorString(e));
      return EBE_ERR_HIP;
    }
  }
  EBE_TRY_HIP(hipStreamSynchronize(s));  // the station list is freed on return
  return worst;
}

ebe_status ebe_invert_lcurve(int32_t n_obs, int32_t n_basis, const double* G, const double* d, int32_t n_reg,
                             const double* L, int32_t n_alpha, const double* alphas_host, double* a, double* rho,
                             double* eta, double* curvature, int32_t* corner, void* stream) {
  if (n_obs < 1 || n_basis < 1 || n_reg < 1 || n_alpha < 1 || !G || !d || !L || !alphas_host || !a || !rho || !eta) {
    set_error("ebe_invert_lcurve: null argument or empty size");
    return EBE_ERR_ARG;
  }
  if (n_basis > kLsqMaxBasis || n_alpha > kLcurveMax) {
    set_error("ebe_invert_lcurve: %d basis functions (at most %d) or %d weights (at most %d)", n_basis,
              kLsqMaxBasis, n_alpha, kLcurveMax);
    return EBE_ERR_ARG;
  }
  if (n_alpha >= 3 && (!curvature || !corner)) {
    set_error("ebe_invert_lcurve: curvature and corner are needed for three or more weights");
    return EBE_ERR_ARG;
  }
  for (int32_t i = 0; i < n_alpha; ++i)
    if (!(alphas_host[i] > 0.0) || !std::isfinite(alphas_host[i]) || (i > 0 && !(alphas_host[i] > alphas_host[i - 1]))) {
      set_error("ebe_invert_lcurve: the weights must be positive, finite and increasing (entry %d)", i);
      return EBE_ERR_ARG;
    }
  const size_t m = size_t(n_obs) + size_t(n_reg);
  DBuf work, alphas;
  ebe_status st = work.alloc(size_t(n_alpha) * m * size_t(n_basis + 1) * sizeof(double));
  if (st == EBE_OK) st = alphas.alloc(size_t(n_alpha) * sizeof(double));
  if (st != EBE_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipMemcpyAsync(alphas.as<void>(), alphas_host, size_t(n_alpha) * sizeof(double),
                                hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = launch_lsq_lcurve(G, d, L, alphas.as<double>(), n_obs, n_reg, n_basis, n_alpha, work.as<double>(), a, rho, eta,
                          curvature, corner, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);  // the workspace is freed on return
  if (e != hipSuccess) {
    set_error("ebe_invert_lcurve: %s", hipGetErrorString(e));
    return EBE_ERR_HIP;
  }
  return EBE_OK;
}

}  // extern "C"
