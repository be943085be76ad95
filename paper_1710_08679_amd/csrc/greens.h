// Internal declarations of the Green's-function pipeline (greens.cpp,
// greens_kernels.hip): the fault handle and the kernel launchers.
#pragma once

#include "ebe_internal.h"

namespace ebe {

constexpr int kLsqMaxBasis = 512;  // basis functions of one inversion (back-substitution LDS)
constexpr int kLcurveMax = 1024;   // regularisation weights of one L-curve

// f = split-node forces of basis functions col0 .. col0 + nrhs - 1 (f zeroed first)
hipError_t launch_split_forces(const ebe_mesh* m, const int32_t* fel, const int8_t* fside, const int32_t* frow,
                               const double* basis, const double* dirs, int32_t nbasis, int32_t nfel, int32_t col0,
                               int32_t nrhs, double* f, hipStream_t s);
// G[3 s + d][col0 + r] = u[st[s]][d][r] for r < nrhs (G has ld columns)
hipError_t launch_gather_obs(const double* u, int32_t nrhs, const int32_t* st, int32_t nst, double* G, int32_t ld,
                             int32_t col0, hipStream_t s);
// Eq. (5) for every alpha (work: nalpha * (nobs + nreg) * (nb + 1) doubles),
// then the L-curve curvature and its corner when nalpha >= 3
hipError_t launch_lsq_lcurve(const double* G, const double* d, const double* L, const double* alphas, int32_t nobs,
                             int32_t nreg, int32_t nb, int32_t nalpha, double* work, double* a, double* rho,
                             double* eta, double* curv, int32_t* corner, hipStream_t s);

}  // namespace ebe

struct ebe_fault {
  ebe_mesh* mesh = nullptr;
  int32_t nbasis = 0, nfel = 0;
  int64_t nfault = 0;
  ebe::DBuf fel;    // int32 [nfel] elements touching the fault
  ebe::DBuf fside;  // int8  [nfel] their side (+1 / -1)
  ebe::DBuf frow;   // int32 [nfel][10] fault-node row of each local node, -1 off the fault
  ebe::DBuf basis;  // double [nfault][nbasis]
  ebe::DBuf dirs;   // double [nbasis][3]
  ebe::DBuf f, u;   // [N][3][16] FP64 load and solution of one set of basis functions
};
