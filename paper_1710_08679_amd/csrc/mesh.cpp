// Mesh handle: validation of the host arrays, derived tables (edge
// end-points, corner -> edge-node adjacency, packed connectivity) and upload.
//
// The handle holds exactly what an EBE product needs to rebuild every element
// matrix on the fly (Section 2, EBE method): connectivity (Q_i), coordinates
// and per-element material.  A mesh from ebe_mesh_create must be
// straight-sided (checked here), so its K_i depends only on the four corners
// and only corner coordinates are kept; one from ebe_mesh_create_curved keeps
// every node's coordinates for the isoparametric element kernel, after
// checking that each element's Jacobian is positive at its quadrature points
// and nodes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "ebe_internal.h"
#include "p2_element.h"

namespace ebe {

static thread_local char g_err[1024] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

ebe_status DBuf::alloc(size_t bytes) {
  if (bytes <= n_ && p_) return EBE_OK;
  release();
  if (bytes == 0) bytes = 1;
  hipError_t e = hipMalloc(&p_, bytes);
  if (e != hipSuccess) {
    p_ = nullptr;
    set_error("hipMalloc(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
    (void)hipGetLastError();
    return EBE_ERR_OOM;
  }
  n_ = bytes;
  return EBE_OK;
}

void DBuf::release() {
  if (p_) (void)hipFree(p_);
  p_ = nullptr;
  n_ = 0;
}

}  // namespace ebe

using namespace ebe;

namespace {

const int kEdge[6][2] = {{0, 1}, {1, 2}, {0, 2}, {0, 3}, {1, 3}, {2, 3}};

template <class T>
ebe_status upload(DBuf& b, const T* host, size_t count, hipStream_t s) {
  ebe_status st = b.alloc(count * sizeof(T));
  if (st != EBE_OK) return st;
  EBE_TRY_HIP(hipMemcpyAsync(b.as<void>(), host, count * sizeof(T), hipMemcpyHostToDevice, s));
  return EBE_OK;
}

bool material_ok(double E, double nu) {
  return std::isfinite(E) && std::isfinite(nu) && E > 0.0 && nu > -1.0 && nu < 0.5;
}

}  // namespace

extern "C" {

const char* ebe_last_error(void) { return g_err; }

const char* ebe_status_string(ebe_status s) {
  switch (s) {
    case EBE_OK: return "ok";
    case EBE_NOT_CONVERGED: return "not converged";
    case EBE_ERR_ARG: return "invalid argument";
    case EBE_ERR_INDEX: return "connectivity index out of range or inconsistent";
    case EBE_ERR_INVERTED: return "inverted or degenerate element";
    case EBE_ERR_CURVED: return "curved element (edge node off the edge midpoint)";
    case EBE_ERR_MATERIAL: return "invalid material";
    case EBE_ERR_OOM: return "device out of memory";
    case EBE_ERR_HIP: return "HIP runtime error";
    case EBE_ERR_BREAKDOWN: return "CG breakdown: operator not positive definite";
    case EBE_ERR_NONFINITE: return "non-finite value";
    case EBE_ERR_NUMBERING: return "numbering is not vertex-first";
    default: return "unknown status";
  }
}

const char* ebe_build_info(void) {
  return "gfx950; HIP; FP32 packed ops disabled; unsafe FP atomics (coarse-grained memory)";
}

static ebe_status create_mesh(const char* fn, bool curved, const double* xyz, int64_t n_nodes,
                              int64_t n_vertices, const int32_t* conn10, int64_t n_elem, const double* young,
                              const double* poisson, const uint8_t* dof_fixed, void* stream, ebe_mesh** out) {
  if (!out) {
    set_error("%s: out is NULL", fn);
    return EBE_ERR_ARG;
  }
  *out = nullptr;
  if (!xyz || !conn10 || !young || !poisson) {
    set_error("%s: null input pointer", fn);
    return EBE_ERR_ARG;
  }
  if (n_nodes <= 0 || n_vertices <= 0 || n_elem <= 0 || n_vertices > n_nodes ||
      n_nodes >= (int64_t(1) << kIdxBits)) {
    set_error("%s: bad sizes n_nodes=%lld n_vertices=%lld n_elem=%lld", fn,
              (long long)n_nodes, (long long)n_vertices, (long long)n_elem);
    return EBE_ERR_ARG;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t N = n_nodes, Nv = n_vertices, E = n_elem, Ne = N - Nv;

  for (int64_t i = 0; i < 3 * N; ++i)
    if (!std::isfinite(xyz[i])) {
      set_error("%s: non-finite coordinate at node %lld", fn, (long long)(i / 3));
      return EBE_ERR_NONFINITE;
    }
  for (int64_t e = 0; e < E; ++e)
    if (!material_ok(young[e], poisson[e])) {
      set_error("%s: element %lld has E=%g nu=%g", fn, (long long)e, young[e], poisson[e]);
      return EBE_ERR_MATERIAL;
    }

  // index range and vertex-first numbering
  std::vector<uint8_t> seen(N, 0);
  for (int64_t e = 0; e < E; ++e) {
    const int32_t* c = conn10 + 10 * e;
    for (int a = 0; a < 10; ++a) {
      if (c[a] < 0 || c[a] >= N) {
        set_error("%s: element %lld node %d index %d out of [0,%lld)", fn, (long long)e, a,
                  c[a], (long long)N);
        return EBE_ERR_INDEX;
      }
      if ((a < 4) != (c[a] < Nv)) {
        set_error("%s: element %lld local node %d (id %d) breaks vertex-first numbering", fn,
                  (long long)e, a, c[a]);
        return EBE_ERR_NUMBERING;
      }
      seen[c[a]] = 1;
    }
  }
  for (int64_t i = 0; i < N; ++i)
    if (!seen[i]) {
      set_error("%s: node %lld is not used by any element", fn, (long long)i);
      return EBE_ERR_INDEX;
    }
  seen.clear();
  seen.shrink_to_fit();

  // edge end-points (consistent across elements), orientation and straightness
  std::vector<int32_t> ends(2 * Ne, -1);
  for (int64_t e = 0; e < E; ++e) {
    const int32_t* c = conn10 + 10 * e;
    const double* x0 = xyz + 3 * c[0];
    double d[3][3];
    for (int k = 0; k < 3; ++k)
      for (int j = 0; j < 3; ++j) d[k][j] = xyz[3 * c[k + 1] + j] - x0[j];
    const double det = d[0][0] * (d[1][1] * d[2][2] - d[1][2] * d[2][1]) -
                       d[0][1] * (d[1][0] * d[2][2] - d[1][2] * d[2][0]) +
                       d[0][2] * (d[1][0] * d[2][1] - d[1][1] * d[2][0]);
    double hmax = 0.0;
    for (int k = 0; k < 6; ++k) {
      const double* xp = xyz + 3 * c[kEdge[k][0]];
      const double* xq = xyz + 3 * c[kEdge[k][1]];
      double l2 = 0.0;
      for (int j = 0; j < 3; ++j) l2 += (xq[j] - xp[j]) * (xq[j] - xp[j]);
      hmax = std::max(hmax, std::sqrt(l2));
    }
    if (!(det > 1e-14 * hmax * hmax * hmax)) {
      set_error("%s: element %lld has det=%g (inverted or degenerate)", fn, (long long)e, det);
      return EBE_ERR_INVERTED;
    }
    if (curved) {
      // the Jacobian of the quadratic map must be positive at the four
      // quadrature points and at the ten nodes
      double dl[10][3];
      for (int a = 0; a < 10; ++a)
        for (int j = 0; j < 3; ++j) dl[a][j] = xyz[3 * c[a] + j] - x0[j];
      for (int pt = 0; pt < 14; ++pt) {
        double L[4] = {0.0, 0.0, 0.0, 0.0};
        if (pt < 4) {
          for (int k = 0; k < 4; ++k) L[k] = quad_l(pt, k);
        } else if (pt < 8) {
          L[pt - 4] = 1.0;
        } else {
          L[kEdge[pt - 8][0]] = L[kEdge[pt - 8][1]] = 0.5;
        }
        double cj[3][3];
        curved_jacobian(dl, L, cj);
        const double dj = det_columns(cj);
        if (!(dj > 1e-14 * hmax * hmax * hmax)) {
          set_error("%s: element %lld has det J = %g at %s %d (inverted or degenerate)", fn, (long long)e, dj,
                    pt < 4 ? "quadrature point" : "node", pt < 4 ? pt : pt - 4);
          return EBE_ERR_INVERTED;
        }
      }
    }
    for (int k = 0; k < 6; ++k) {
      int32_t p = c[kEdge[k][0]], q = c[kEdge[k][1]];
      const double* xm = xyz + 3 * c[4 + k];
      double dev = 0.0;
      for (int j = 0; j < 3; ++j) {
        double mid = 0.5 * (xyz[3 * p + j] + xyz[3 * q + j]);
        dev = std::max(dev, std::fabs(xm[j] - mid));
      }
      if (!curved && dev > 1e-10 * hmax) {
        set_error("%s: element %lld edge %d node is %g off the midpoint", fn, (long long)e, k, dev);
        return EBE_ERR_CURVED;
      }
      if (p > q) std::swap(p, q);
      int32_t* en = &ends[2 * (int64_t(c[4 + k]) - Nv)];
      if (en[0] < 0) {
        en[0] = p;
        en[1] = q;
      } else if (en[0] != p || en[1] != q) {
        set_error("%s: edge node %d has end points (%d,%d) and (%d,%d)", fn, c[4 + k], en[0],
                  en[1], p, q);
        return EBE_ERR_INDEX;
      }
    }
  }

  // corner -> incident edge nodes (CSR), for the restriction P1^T
  std::vector<int32_t> off(Nv + 1, 0), idx(2 * Ne);
  for (int64_t k = 0; k < Ne; ++k) {
    off[ends[2 * k] + 1]++;
    off[ends[2 * k + 1] + 1]++;
  }
  for (int64_t v = 0; v < Nv; ++v) off[v + 1] += off[v];
  {
    std::vector<int32_t> fill(off.begin(), off.end() - 1);
    for (int64_t k = 0; k < Ne; ++k) {
      idx[fill[ends[2 * k]]++] = int32_t(Nv + k);
      idx[fill[ends[2 * k + 1]]++] = int32_t(Nv + k);
    }
  }

  // corner -> incident elements (CSR, by element), for the row-wise K1 assembly
  if (4 * E >= (int64_t(1) << 31)) {
    set_error("%s: too many elements for 32-bit corner incidence lists", fn);
    return EBE_ERR_ARG;
  }
  std::vector<int32_t> veoff(Nv + 1, 0), vel(size_t(4 * E));
  for (int64_t e = 0; e < E; ++e)
    for (int a = 0; a < 4; ++a) veoff[conn10[10 * e + a] + 1]++;
  for (int64_t v = 0; v < Nv; ++v) veoff[v + 1] += veoff[v];
  {
    std::vector<int32_t> fill(veoff.begin(), veoff.end() - 1);
    for (int64_t e = 0; e < E; ++e)
      for (int a = 0; a < 4; ++a) vel[fill[conn10[10 * e + a]]++] = int32_t(4 * e + a);
  }

  // node fix bits and packed connectivity
  std::vector<uint8_t> fix(N, 0);
  bool any_bc = false;
  if (dof_fixed) {
    for (int64_t i = 0; i < N; ++i) {
      uint8_t b = 0;
      for (int c = 0; c < 3; ++c)
        if (dof_fixed[3 * i + c]) b |= uint8_t(1u << c);
      fix[i] = b;
      any_bc |= (b != 0);
    }
  }
  // rows of the assembled linear-level operator: row v holds v and the far
  // ends of its incident edges, increasing (the corner graph's edges are the
  // edge nodes)
  std::vector<int32_t> bptr(Nv + 1, 0), bcol;
  bcol.reserve(size_t(Nv + 2 * Ne));
  for (int64_t v = 0; v < Nv; ++v) {
    const size_t b0 = bcol.size();
    bcol.push_back(int32_t(v));
    for (int32_t k = off[v]; k < off[v + 1]; ++k) {
      const int64_t ed = idx[k] - Nv;
      bcol.push_back(ends[2 * ed] == v ? ends[2 * ed + 1] : ends[2 * ed]);
    }
    std::sort(bcol.begin() + b0, bcol.end());
    bcol.erase(std::unique(bcol.begin() + b0, bcol.end()), bcol.end());
    if (bcol.size() >= size_t(1) << 31) {
      set_error("%s: corner graph too large for 32-bit block indices", fn);
      return EBE_ERR_ARG;
    }
    bptr[v + 1] = int32_t(bcol.size());
  }
  // sliced layout of K1 (padding: zero blocks in the row's own column) and level 2
  std::vector<int32_t> soff, scol;
  {
    const ebe_status sst = slice_rows(bptr, bcol, fix.data(), soff, scol);
    if (sst != EBE_OK) return sst;
  }

  std::vector<int32_t> packed(10 * E);
  for (int64_t k = 0; k < 10 * E; ++k) packed[k] = conn10[k] | (int32_t(fix[conn10[k]]) << kIdxBits);

  // corner coordinates (curved meshes: every node's, corners first)
  const int64_t Nx = curved ? N : Nv;
  std::vector<double> xv(4 * Nx);
  for (int64_t v = 0; v < Nx; ++v) {
    xv[4 * v + 0] = xyz[3 * v + 0];
    xv[4 * v + 1] = xyz[3 * v + 1];
    xv[4 * v + 2] = xyz[3 * v + 2];
    xv[4 * v + 3] = 0.0;
  }

  ebe_mesh* m = new (std::nothrow) ebe_mesh();
  if (!m) {
    set_error("%s: host allocation failed", fn);
    return EBE_ERR_OOM;
  }
  m->n_nodes = N;
  m->n_vertices = Nv;
  m->n_elem = E;
  m->has_bc = any_bc;
  m->curved = curved;
  (void)hipGetDevice(&m->device);
  ebe_status st = EBE_OK;
  if (st == EBE_OK) st = upload(m->conn, packed.data(), packed.size(), s);
  if (st == EBE_OK) st = upload(m->xv, xv.data(), xv.size(), s);
  if (st == EBE_OK) st = upload(m->young, young, size_t(E), s);
  if (st == EBE_OK) st = upload(m->poisson, poisson, size_t(E), s);
  if (st == EBE_OK) st = upload(m->fix, fix.data(), fix.size(), s);
  if (st == EBE_OK) st = upload(m->edge_ends, ends.data(), std::max<size_t>(ends.size(), 1), s);
  if (st == EBE_OK) st = upload(m->v2e_off, off.data(), off.size(), s);
  if (st == EBE_OK) st = upload(m->v2e_idx, idx.data(), std::max<size_t>(idx.size(), 1), s);
  if (st == EBE_OK) st = upload(m->v2el_off, veoff.data(), veoff.size(), s);
  if (st == EBE_OK) st = upload(m->v2el, vel.data(), vel.size(), s);
  if (st == EBE_OK) st = upload_asm(m->k1, Nv, soff, scol, s);
  if (st == EBE_OK) st = build_level2(m, bptr, bcol, fix.data(), s);
  if (st == EBE_OK) st = m->lame64.alloc(size_t(E) * 2 * sizeof(double));
  if (st == EBE_OK) st = m->lame32.alloc(size_t(E) * 2 * sizeof(float));
  if (st == EBE_OK) st = build_patches(m, conn10, fix.data(), s);
  if (st == EBE_OK) st = m->gacc.alloc(kGammaBytes);
  if (st == EBE_OK) {
    hipError_t he = launch_lame(m, s);
    if (he == hipSuccess) he = launch_fill_zero(m->gacc.as<void>(), kGammaBytes, s);
    if (he == hipSuccess) he = hipStreamSynchronize(s);
    if (he != hipSuccess) {
      set_error("%s: upload failed: %s", fn, hipGetErrorString(he));
      st = EBE_ERR_HIP;
    }
  }
  if (st != EBE_OK) {
    delete m;
    return st;
  }
  *out = m;
  return EBE_OK;
}

ebe_status ebe_mesh_create(const double* xyz, int64_t n_nodes, int64_t n_vertices, const int32_t* conn10,
                           int64_t n_elem, const double* young, const double* poisson, const uint8_t* dof_fixed,
                           void* stream, ebe_mesh** out) {
  return create_mesh("ebe_mesh_create", false, xyz, n_nodes, n_vertices, conn10, n_elem, young, poisson, dof_fixed,
                     stream, out);
}

ebe_status ebe_mesh_create_curved(const double* xyz, int64_t n_nodes, int64_t n_vertices, const int32_t* conn10,
                                  int64_t n_elem, const double* young, const double* poisson,
                                  const uint8_t* dof_fixed, void* stream, ebe_mesh** out) {
  return create_mesh("ebe_mesh_create_curved", true, xyz, n_nodes, n_vertices, conn10, n_elem, young, poisson,
                     dof_fixed, stream, out);
}

ebe_status ebe_mesh_set_material(ebe_mesh* m, const double* young_dev, const double* poisson_dev,
                                 void* stream) {
  if (!m || !young_dev || !poisson_dev) {
    set_error("ebe_mesh_set_material: null argument");
    return EBE_ERR_ARG;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t bytes = size_t(m->n_elem) * sizeof(double);
  ebe_status st = m->ws.flags.alloc(64 * sizeof(int));
  if (st != EBE_OK) return st;
  int* bad = m->ws.flags.as<int>();
  EBE_TRY_HIP(launch_check_material(young_dev, poisson_dev, m->n_elem, bad, s));
  int hbad = 0;
  EBE_TRY_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s));
  EBE_TRY_HIP(hipStreamSynchronize(s));
  if (hbad) {
    set_error("ebe_mesh_set_material: %d elements with E <= 0 or nu outside (-1, 0.5)", hbad);
    return EBE_ERR_MATERIAL;
  }
  EBE_TRY_HIP(hipMemcpyAsync(m->young.as<void>(), young_dev, bytes, hipMemcpyDeviceToDevice, s));
  EBE_TRY_HIP(hipMemcpyAsync(m->poisson.as<void>(), poisson_dev, bytes, hipMemcpyDeviceToDevice, s));
  EBE_TRY_HIP(launch_lame(m, s));
  m->minv_ready = false;
  m->geo_ready[0] = m->geo_ready[1] = false;
  m->k1.ready[0] = m->k1.ready[1] = m->k1.ready16 = false;
  m->a2.ready[0] = m->a2.ready[1] = m->a2.ready16 = false;
  return EBE_OK;
}

ebe_status ebe_mesh_info(const ebe_mesh* m, int64_t* n_nodes, int64_t* n_vertices, int64_t* n_elem) {
  if (!m) {
    set_error("ebe_mesh_info: null mesh");
    return EBE_ERR_ARG;
  }
  if (n_nodes) *n_nodes = m->n_nodes;
  if (n_vertices) *n_vertices = m->n_vertices;
  if (n_elem) *n_elem = m->n_elem;
  return EBE_OK;
}

void ebe_mesh_destroy(ebe_mesh* m) {
  if (!m) return;
  if (m->ws.host_flags) (void)hipHostFree(m->ws.host_flags);
  for (auto& g : m->ws.graphs) (void)hipGraphExecDestroy(g.exec);
  delete m;
}

}  // extern "C"
