// Element operators of tetrahedra, applied without forming the element
// matrix (Section 2, EBE method: K_i is rebuilt from the node coordinates and
// the material at every product): straight-sided elements in closed form
// (p2_apply, p1_apply), curved isoparametric ones by quadrature (p2c_apply).
//
// Quadratic (10-node) element.  With barycentric coordinates L_k and their
// constant gradients G_k, the displacement gradient of a quadratic field is
// linear in L:  grad u = sum_k L_k H_k  with
//     H_k = 4 sum_{m != k} (u_{km} - u_k) (x) G_m  -  sum_{i>=1} (u_i - u_0) (x) G_i,
// where u_{km} is the edge node between corners k and m.  The stress is
// sigma = sum_k L_k S_k with S_k = lambda tr(H_k) I + 2 mu sym(H_k), and
// int L_k L_l dV = V (1 + delta_kl) / 20 turns the nodal forces
// f_a = int sigma grad N_a dV into
//     corner i:        f_i  = (4 S'_i - S') G_i
//     edge (k, m):     f_km = 4 [(S'_m + S') G_k + (S'_k + S') G_m]
// with S'_k = (V/20) S_k and S' = sum_k S'_k.  This equals K_e u_e of the
// isoparametric B^T D B integral exactly (to rounding) for straight elements.
//
// Symmetric tensors are stored as (xx, yy, zz, yz, zx, xy); strains carry
// engineering shears (yz = du_y/dz + du_z/dy).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ebe {

#define EBE_HD __host__ __device__ __forceinline__

// local node of the edge between corners k != m (VTK quadratic-tetra order:
// edges (0,1), (1,2), (0,2), (0,3), (1,3), (2,3) are local nodes 4..9)
EBE_HD constexpr int edge_node(int k, int m) {
  const int a = k < m ? k : m, b = k < m ? m : k;
  return a == 0 ? (b == 1 ? 4 : (b == 2 ? 6 : 7)) : (a == 1 ? (b == 2 ? 5 : 8) : 9);
}
EBE_HD constexpr int edge_end(int q, int side) {
  return side == 0 ? (q == 0 ? 0 : q == 1 ? 1 : q == 2 ? 0 : q == 3 ? 0 : q == 4 ? 1 : 2)
                   : (q == 0 ? 1 : q == 1 ? 2 : q == 2 ? 2 : 3);
}

// Barycentric gradients G[4][3] and volume of the corner tetrahedron.  Edge
// vectors are formed in FP64 (coordinates are FP64), the rest in T.
template <typename T>
EBE_HD T tet_geometry(const double4& p0, const double4& p1, const double4& p2,
                                          const double4& p3, T G[4][3]) {
  const T a0 = T(p1.x - p0.x), a1 = T(p1.y - p0.y), a2 = T(p1.z - p0.z);
  const T b0 = T(p2.x - p0.x), b1 = T(p2.y - p0.y), b2 = T(p2.z - p0.z);
  const T c0 = T(p3.x - p0.x), c1 = T(p3.y - p0.y), c2 = T(p3.z - p0.z);
  // rows of the inverse Jacobian: (b x c, c x a, a x b) / det
  const T bc0 = b1 * c2 - b2 * c1, bc1 = b2 * c0 - b0 * c2, bc2 = b0 * c1 - b1 * c0;
  const T ca0 = c1 * a2 - c2 * a1, ca1 = c2 * a0 - c0 * a2, ca2 = c0 * a1 - c1 * a0;
  const T ab0 = a1 * b2 - a2 * b1, ab1 = a2 * b0 - a0 * b2, ab2 = a0 * b1 - a1 * b0;
  const T det = a0 * bc0 + a1 * bc1 + a2 * bc2;
  const T inv = T(1) / det;
  G[1][0] = bc0 * inv; G[1][1] = bc1 * inv; G[1][2] = bc2 * inv;
  G[2][0] = ca0 * inv; G[2][1] = ca1 * inv; G[2][2] = ca2 * inv;
  G[3][0] = ab0 * inv; G[3][1] = ab1 * inv; G[3][2] = ab2 * inv;
#pragma unroll
  for (int d = 0; d < 3; ++d) G[0][d] = -(G[1][d] + G[2][d] + G[3][d]);
  return det * T(1.0 / 6.0);
}

// w += engineering strain of the outer product d (x) g
template <typename T>
EBE_HD void acc_eng(T w[6], const T d[3], const T g[3]) {
  w[0] += d[0] * g[0];
  w[1] += d[1] * g[1];
  w[2] += d[2] * g[2];
  w[3] += d[1] * g[2] + d[2] * g[1];
  w[4] += d[2] * g[0] + d[0] * g[2];
  w[5] += d[0] * g[1] + d[1] * g[0];
}

// out = P g for symmetric P
template <typename T>
EBE_HD void sym_mv(const T P[6], const T g[3], T out[3]) {
  out[0] = P[0] * g[0] + P[5] * g[1] + P[4] * g[2];
  out[1] = P[5] * g[0] + P[1] * g[1] + P[3] * g[2];
  out[2] = P[4] * g[0] + P[3] * g[1] + P[2] * g[2];
}

// stress (scaled) from engineering strain: cl = lambda * s, cm = mu * s
template <typename T>
EBE_HD void stress(const T e[6], T cl, T cm, T S[6]) {
  const T tr = e[0] + e[1] + e[2];
  const T cm2 = cm + cm;
  S[0] = cl * tr + cm2 * e[0];
  S[1] = cl * tr + cm2 * e[1];
  S[2] = cl * tr + cm2 * e[2];
  S[3] = cm * e[3];
  S[4] = cm * e[4];
  S[5] = cm * e[5];
}

// w = engineering strain of d (x) g (one multiply per product, the second
// product of each shear pair fused)
template <typename T>
EBE_HD void set_eng(T w[6], const T d[3], const T g[3]) {
  w[0] = d[0] * g[0];
  w[1] = d[1] * g[1];
  w[2] = d[2] * g[2];
  w[3] = d[1] * g[2];
  w[3] += d[2] * g[1];
  w[4] = d[2] * g[0];
  w[4] += d[0] * g[2];
  w[5] = d[0] * g[1];
  w[5] += d[1] * g[0];
}

// w += engineering strain of d (x) g, as nine fused multiply-adds
template <typename T>
EBE_HD void fma_eng(T w[6], const T d[3], const T g[3]) {
  w[0] += d[0] * g[0];
  w[1] += d[1] * g[1];
  w[2] += d[2] * g[2];
  w[3] += d[1] * g[2];
  w[3] += d[2] * g[1];
  w[4] += d[2] * g[0];
  w[4] += d[0] * g[2];
  w[5] += d[0] * g[1];
  w[5] += d[1] * g[0];
}

// out += P g for symmetric P
template <typename T>
EBE_HD void sym_mv_acc(const T P[6], const T g[3], T out[3]) {
  out[0] += P[0] * g[0];
  out[0] += P[5] * g[1];
  out[0] += P[4] * g[2];
  out[1] += P[5] * g[0];
  out[1] += P[1] * g[1];
  out[1] += P[3] * g[2];
  out[2] += P[4] * g[0];
  out[2] += P[3] * g[1];
  out[2] += P[2] * g[2];
}

// f = K_e u for a straight 10-node tetrahedron; cl = lambda V / 20, cm = mu V / 20.
//
// Written with H_k = 4 (V_k + sum_{m != k} E_km) - sum_i V_i, V_i = u_i (x) G_i
// and E_km = u_{km} (x) G_m (using G_k = -sum_{m != k} G_m), which needs 16
// outer products and no differences; every accumulation is a fused
// multiply-add.  About 440 floating-point instructions per element and case.
//
// Streaming form: u(a, c) returns component c of local node a and is called
// once per node and component while the strains are accumulated (an edge
// node's value feeds both of its corners' strains at once); emit(a, f) takes
// the force of node a as soon as it is known.  Only the 30 strain sums (then
// the 30 stresses) and the gradients stay live, never all 30 nodal values.
//
// with_energy: energy = u_eᵀ K_e u_e = int sigma : eps dV, formed from
// the strains e_k = 4 w_k - A and scaled stresses as
//     sum_k S'_k : e_k + S' : sum_k e_k
// (int L_k L_l dV = V (1 + delta_kl) / 20; engineering shears pair with the
// shear stresses), so the nodal values need not be kept for it.
template <typename T, class U, class Emit>
EBE_HD void p2_apply(const T G[4][3], T cl, T cm, U&& u, Emit&& emit, bool with_energy, T& energy) {
  T w[4][6];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const T ui[3] = {u(i, 0), u(i, 1), u(i, 2)};
    set_eng(w[i], ui, G[i]);
  }
  T A[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) A[c] = (w[0][c] + w[1][c]) + (w[2][c] + w[3][c]);
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    const int k = edge_end(q, 0), m = edge_end(q, 1);
    const T ue[3] = {u(4 + q, 0), u(4 + q, 1), u(4 + q, 2)};
    fma_eng(w[k], ue, G[m]);
    fma_eng(w[m], ue, G[k]);
  }
  // S'_k from the strain 4 w_k - A (w is overwritten by S'_k)
  T Ssum[6], esum[6];
  T en = T(0);
  const T cm2 = cm + cm;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    T e[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) e[c] = T(4) * w[k][c] - A[c];
    const T clt = cl * ((e[0] + e[1]) + e[2]);
    w[k][0] = cm2 * e[0] + clt;
    w[k][1] = cm2 * e[1] + clt;
    w[k][2] = cm2 * e[2] + clt;
    w[k][3] = cm * e[3];
    w[k][4] = cm * e[4];
    w[k][5] = cm * e[5];
#pragma unroll
    for (int c = 0; c < 6; ++c) Ssum[c] = (k == 0) ? w[k][c] : Ssum[c] + w[k][c];
    if (with_energy) {
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        en += w[k][c] * e[c];
        esum[c] = (k == 0) ? e[c] : esum[c] + e[c];
      }
    }
  }
  if (with_energy) {
#pragma unroll
    for (int c = 0; c < 6; ++c) en += Ssum[c] * esum[c];
    energy = en;
  }
  // corners: f_i = (4 S'_i - S') G_i
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    T P[6], f[3];
#pragma unroll
    for (int c = 0; c < 6; ++c) P[c] = T(4) * w[i][c] - Ssum[c];
    sym_mv(P, G[i], f);
    emit(i, f);
  }
  // edges: f_km = T'_m G_k + T'_k G_m with T'_k = 4 (S'_k + S')
  T S4[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) S4[c] = T(4) * Ssum[c];
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int c = 0; c < 6; ++c) w[k][c] = T(4) * w[k][c] + S4[c];
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    const int k = edge_end(q, 0), m = edge_end(q, 1);
    T f[3];
    sym_mv(w[m], G[k], f);
    sym_mv_acc(w[k], G[m], f);
    emit(4 + q, f);
  }
}

template <typename T>
EBE_HD void p2_forces(const T G[4][3], T cl, T cm, const T u[10][3], T f[10][3]) {
  T unused = T(0);
  p2_apply<T>(
      G, cl, cm, [&](int a, int c) { return u[a][c]; },
      [&](int a, const T fa[3]) {
        f[a][0] = fa[0];
        f[a][1] = fa[1];
        f[a][2] = fa[2];
      },
      false, unused);
}

// f = K1_e u for a 4-node tetrahedron (constant strain); cl = lambda V, cm = mu V.
// with_energy: energy = u_eᵀ K1_e u_e = S : e (V already in cl, cm).
template <typename T, class U, class Emit>
EBE_HD void p1_apply(const T G[4][3], T cl, T cm, U&& u, Emit&& emit, bool with_energy, T& energy) {
  const T u0[3] = {u(0, 0), u(0, 1), u(0, 2)};
  T e6[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
#pragma unroll
  for (int i = 1; i < 4; ++i) {
    const T d[3] = {u(i, 0) - u0[0], u(i, 1) - u0[1], u(i, 2) - u0[2]};
    acc_eng(e6, d, G[i]);
  }
  T S[6];
  stress(e6, cl, cm, S);
  if (with_energy) {
    T en = T(0);
#pragma unroll
    for (int c = 0; c < 6; ++c) en += S[c] * e6[c];
    energy = en;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    T f[3];
    sym_mv(S, G[i], f);
    emit(i, f);
  }
}

template <typename T>
EBE_HD void p1_forces(const T G[4][3], T cl, T cm, const T u[4][3], T f[4][3]) {
  T unused = T(0);
  p1_apply<T>(
      G, cl, cm, [&](int a, int c) { return u[a][c]; },
      [&](int a, const T fa[3]) {
        f[a][0] = fa[0];
        f[a][1] = fa[1];
        f[a][2] = fa[2];
      },
      false, unused);
}

// ---------------------------------------------------------------------------
// Curved (isoparametric) 10-node tetrahedra: edge nodes anywhere, the element
// map x(L) = sum_a N_a(L) x_a quadratic, its Jacobian varying inside the
// element.  K_e = sum_q w_q B_q^T D B_q det J_q with the symmetric 4-point
// rule (exact for straight elements, where this equals p2_apply to
// rounding): point q has barycentric coordinate kQa at corner q and kQb at
// the other three, weight 1/24 (a quarter of the reference volume 1/6);
// kQa = (5 + 3 sqrt 5) / 20, kQb = (5 - sqrt 5) / 20.
//
// Derivatives are taken with the four barycentric coordinates as independent
// variables: dN_i/dL_k = (4 L_i - 1) delta_ik for corner i, and for the edge
// node between corners k and m dN_km/dL_k = 4 L_m.  With G_k = grad L_k
// (G_0 = -(G_1 + G_2 + G_3)), grad N_a = sum_k (dN_a/dL_k) G_k, so a field
// sum_a v_a N_a has the gradient sum_k V_k (x) G_k with
//     V_k = sum_a v_a dN_a/dL_k = (4 L_k - 1) v_k + 4 sum_{m != k} L_m v_km.
// Applied to the coordinates this gives the Jacobian's columns
// dx/dL_j - dx/dL_0 = X_j - X_0 (j = 1..3), whose inverse's rows are
// G_1..G_3; applied to a displacement it gives grad u.
// ---------------------------------------------------------------------------
constexpr double kQa = (5.0 + 3.0 * 2.23606797749978969641) / 20.0;
constexpr double kQb = (5.0 - 2.23606797749978969641) / 20.0;

// barycentric coordinate of corner k at quadrature point q
EBE_HD constexpr double quad_l(int q, int k) { return q == k ? kQa : kQb; }

// Columns c[j] = X_{j+1} - X_0 of the Jacobian at barycentric point L, from
// the node coordinates relative to corner 0 (d[0] = 0).
EBE_HD void curved_jacobian(const double d[10][3], const double L[4], double c[3][3]) {
  double X[4][3];
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int i = 0; i < 3; ++i) X[k][i] = (4.0 * L[k] - 1.0) * d[k][i];
#pragma unroll
  for (int e = 0; e < 6; ++e) {
    const int k = edge_end(e, 0), m = edge_end(e, 1);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      X[k][i] += 4.0 * L[m] * d[4 + e][i];
      X[m][i] += 4.0 * L[k] * d[4 + e][i];
    }
  }
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int i = 0; i < 3; ++i) c[j][i] = X[j + 1][i] - X[0][i];
}

// det of the Jacobian with columns c
EBE_HD double det_columns(const double c[3][3]) {
  return c[0][0] * (c[1][1] * c[2][2] - c[1][2] * c[2][1]) + c[0][1] * (c[1][2] * c[2][0] - c[1][0] * c[2][2]) +
         c[0][2] * (c[1][0] * c[2][1] - c[1][1] * c[2][0]);
}

// Gradients G[j] = grad L_{j+1} (j = 0..2) at quadrature point q and det J
// there, in FP64, from node coordinates relative to corner 0.
EBE_HD double curved_point(const double d[10][3], int q, double G[3][3]) {
  const double L[4] = {quad_l(q, 0), quad_l(q, 1), quad_l(q, 2), quad_l(q, 3)};
  double c[3][3];
  curved_jacobian(d, L, c);
  // rows of the inverse: (c1 x c2, c2 x c0, c0 x c1) / det
  const double det = det_columns(c);
  const double inv = 1.0 / det;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const double* a = c[(j + 1) % 3];
    const double* b = c[(j + 2) % 3];
    G[j][0] = (a[1] * b[2] - a[2] * b[1]) * inv;
    G[j][1] = (a[2] * b[0] - a[0] * b[2]) * inv;
    G[j][2] = (a[0] * b[1] - a[1] * b[0]) * inv;
  }
  return det;
}

// f = K_e u for a curved 10-node tetrahedron.  geo(q, i) returns the point
// data of quadrature point q: i = 3 j + d (j, d < 3) component d of
// grad L_{j+1}; i = 9: lambda det J_q / 24; i = 10: mu det J_q / 24 (read
// where used, so they need not stay in registers).  u(a, c) is called once
// per node and component, emit(a, f) once per node after all four points.
// with_energy: energy = u_eᵀ K_e u_e = sum_q S_q : e_q (the scaled stress
// against the engineering strain).
template <typename T, class Geo, class U, class Emit>
EBE_HD void p2c_apply(Geo&& geo, U&& u, Emit&& emit, bool with_energy, T& energy) {
  T uc[4][3], ue[6][3], sm[4][3];
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      uc[k][c] = u(k, c);
      sm[k][c] = T(0);
    }
#pragma unroll
  for (int e = 0; e < 6; ++e) {
    const int k = edge_end(e, 0), m = edge_end(e, 1);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      ue[e][c] = u(4 + e, c);
      sm[k][c] += ue[e][c];  // sum over the edge nodes at corner k
      sm[m][c] += ue[e][c];
    }
  }
  const T a4 = T(4.0 * kQa - 1.0), b4 = T(4.0 * kQb - 1.0), bb = T(4.0 * kQb), ab = T(4.0 * (kQa - kQb));
  T S[4][6];
  T en = T(0);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    // V_k = (4 L_k - 1) u_k + 4 kQb sum_{m != k} u_km + 4 (kQa - kQb) u_kq
    T V[4][3];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        V[k][c] = (k == q ? a4 : b4) * uc[k][c] + bb * sm[k][c];
        if (k != q) V[k][c] += ab * ue[edge_node(k, q) - 4][c];
      }
    // grad u: H[c][d] = sum_j (V_j - V_0)[c] G_j[d]
    T Gp[3][3];
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int dd = 0; dd < 3; ++dd) Gp[j][dd] = geo(q, 3 * j + dd);
    T H[3][3];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int dd = 0; dd < 3; ++dd) {
        T h = (V[1][c] - V[0][c]) * Gp[0][dd];
        h += (V[2][c] - V[0][c]) * Gp[1][dd];
        h += (V[3][c] - V[0][c]) * Gp[2][dd];
        H[c][dd] = h;
      }
    const T e6[6] = {H[0][0], H[1][1], H[2][2], H[1][2] + H[2][1], H[2][0] + H[0][2], H[0][1] + H[1][0]};
    stress(e6, geo(q, 9), geo(q, 10), S[q]);
    if (with_energy) {
#pragma unroll
      for (int c = 0; c < 6; ++c) en += S[q][c] * e6[c];
    }
  }
  if (with_energy) energy = en;
  // f_a = sum_q S_q grad N_a(q) = sum_q sum_k (dN_a/dL_k)(q) t_kq, t_kq = S_q G_k(q)
  T f[10][3];
#pragma unroll
  for (int a = 0; a < 10; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) f[a][c] = T(0);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    T t[4][3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const T g[3] = {geo(q, 3 * j), geo(q, 3 * j + 1), geo(q, 3 * j + 2)};
      sym_mv(S[q], g, t[j + 1]);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) t[0][c] = -((t[1][c] + t[2][c]) + t[3][c]);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const T ck = T(4.0 * quad_l(q, k) - 1.0);
#pragma unroll
      for (int c = 0; c < 3; ++c) f[k][c] += ck * t[k][c];
    }
#pragma unroll
    for (int e = 0; e < 6; ++e) {
      const int k = edge_end(e, 0), m = edge_end(e, 1);
      const T lm = T(4.0 * quad_l(q, m)), lk = T(4.0 * quad_l(q, k));
#pragma unroll
      for (int c = 0; c < 3; ++c) f[4 + e][c] += lm * t[k][c] + lk * t[m][c];
    }
  }
#pragma unroll
  for (int a = 0; a < 10; ++a) emit(a, f[a]);
}

}  // namespace ebe
