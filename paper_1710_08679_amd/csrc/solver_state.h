// Device-resident scalars of the multi-case CG loops of Algorithm 1.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "ebe.h"

namespace ebe {

struct InnerScalars {          // Algorithm 1(b), one set per level
  double nr2[EBE_MAX_RHS];     // ||r_j||^2 of the inner right-hand side
  double rho_a[EBE_MAX_RHS];    // (M^-1 e, e) of the current step
  double gamma[EBE_MAX_RHS];    // (p, K p), accumulated by the product that forms q
  double alpha[EBE_MAX_RHS];
  double beta[EBE_MAX_RHS];
  int active;                  // 1 while max_j ||e_j||^2/||r_j||^2 > eps and i < N
  int i;                       // the loop counter of Algorithm 1(b), starts at 1
  long long steps;             // total steps taken (statistics)
};

struct SolverScalars {         // Algorithm 1(a)
  double nf2[EBE_MAX_RHS];     // ||f_j||^2
  double rr[EBE_MAX_RHS];      // ||r_j||^2
  double rel[EBE_MAX_RHS];     // ||r_j|| / ||f_j||
  double rho[EBE_MAX_RHS];
  double alpha[EBE_MAX_RHS];
  double beta[EBE_MAX_RHS];
  double gamma[EBE_MAX_RHS];     // (p, K p), accumulated by the product that forms q
  double max_rel;
  int outer_active;            // 1 while max_j rel_j > tol and iterations remain
  int outer_iter;
  int err;                     // EBE_ERR_BREAKDOWN / EBE_ERR_NONFINITE raised on the device
  int pad;
  InnerScalars inner[3];
};

struct SolverState {
  SolverScalars* sc = nullptr;   // device
  void* partials = nullptr;      // device, per-workgroup partial sums
  unsigned* counter = nullptr;   // device, arrival counter of the last-workgroup reductions
};

// launchers (solver_kernels.hip)
hipError_t sk_mask_u(const ebe_mesh* m, double* u, int nr, SolverState& st, hipStream_t s);
hipError_t sk_outer_init(const ebe_mesh* m, const double* f, const double* q, double* r, int nr, double tol,
                         SolverState& st, hipStream_t s);
// z = M^-1 r (PCGE) or z = u_bar (MG2) is formed where it is used and never stored:
// the z kernels sum (z, q) and (z, r) and set beta; the p kernels form p = z + beta p.
hipError_t sk_outer_z_bj(const ebe_mesh* m, const double* r, const double* q, int nr, SolverState& st,
                         hipStream_t s);
template <typename T>
hipError_t sk_outer_z_cast(const ebe_mesh* m, const T* ub, const double* r, const double* q, int nr,
                           SolverState& st, hipStream_t s);
hipError_t sk_outer_p_bj(const ebe_mesh* m, const double* r, double* p, int nr, SolverState& st, hipStream_t s);
template <typename T>
hipError_t sk_outer_p_cast(const ebe_mesh* m, const T* ub, double* p, int nr, SolverState& st, hipStream_t s);
hipError_t sk_outer_update(const ebe_mesh* m, double* r, double* u, const double* q, const double* p, int nr,
                           double tol, int max_outer, SolverState& st, hipStream_t s);
// the same, also forming the next PCGE step's z sums and beta (z = M^-1 r)
hipError_t sk_outer_update_z_bj(const ebe_mesh* m, double* r, double* u, const double* q, const double* p, int nr,
                                double tol, int max_outer, SolverState& st, hipStream_t s);
template <typename T>
hipError_t sk_cast_bj(const ebe_mesh* m, const double* r, T* rb, T* ub, int nr, SolverState& st, hipStream_t s);
template <typename T>
hipError_t sk_inner_init(const ebe_mesh* m, int level, const T* r, const T* q, T* e, int nr, double eps, int nmax,
                         SolverState& st, hipStream_t s);
template <typename T>
hipError_t sk_inner_p(const ebe_mesh* m, int level, const T* e, T* p, T* q, int nr, SolverState& st,
                      hipStream_t s);
template <typename T>
hipError_t sk_inner_update(const ebe_mesh* m, int level, T* e, T* u, const T* q, const T* p, int nr, double eps,
                           int nmax, SolverState& st, hipStream_t s);
// gamma[j] = (a_j, b_j) on level `level` (rows of that level), summed in a
// fixed order; skipped when gate is non-null and *gate == 0
template <typename T>
hipError_t sk_dot(const ebe_mesh* m, int level, const T* a, const T* b, int nr, double* gamma, const int* gate,
                  SolverState& st, hipStream_t s);

}  // namespace ebe
