// Launchers of the Schur-complement solver's kernels (kernels_schur.hip), used by schur.cpp.
#pragma once

#include "internal.h"

namespace td {

hipError_t launch_schur_interior_coeffs(double* Ai, double* Bi, double* Ci, const double* A, const double* B,
                                        const double* C, const int64_t* intcol, int64_t Nint, int M, hipStream_t st);
hipError_t launch_schur_scatter(double* T, int64_t ldt, const double* base, int64_t ldb, const double* V, int64_t ldv,
                                const double* A, const double* B, const int64_t* intcol, const int32_t* lif,
                                const int32_t* rif, int64_t Nint, int M, int K, double sgn, hipStream_t st);
hipError_t launch_schur_gather(double* out, int64_t ldo, const double* base, int64_t ldb, const double* V, int64_t ldv,
                               const double* Y, int64_t ldy, const double* A, const double* B, const double* C,
                               const int64_t* icol, const int64_t* ileft, const int64_t* iright, int64_t nif, int M,
                               int64_t nGp, int K, int withC, hipStream_t st);
hipError_t launch_schur_assemble(double* X, int64_t ldx, const double* Y, int64_t ldy, const double* xG, int64_t ldg,
                                 const int64_t* intcol, const int64_t* icol, int64_t Nint, int64_t nif, int M, int K,
                                 hipStream_t st);
int schur_dot_parts(int64_t n);
hipError_t launch_coldot(double* d, double* part, const double* x, const double* y, int64_t ld, int64_t n, int K,
                         hipStream_t st);
hipError_t launch_cg_alpha(double* alpha, const double* rz, const double* pq, const int32_t* active, int K,
                           hipStream_t st);
hipError_t launch_cg_update(double* x, double* r, const double* p, const double* q, const double* alpha, int64_t ld,
                            int64_t n, int K, hipStream_t st);
hipError_t launch_cg_direction(double* p, const double* z, const double* rz_new, const double* rz_old,
                               const int32_t* active, int64_t ld, int64_t n, int K, hipStream_t st);
hipError_t launch_cg_status(int32_t* active, double* stat, const double* rr, const double* gg, double tol, int K,
                            hipStream_t st);
hipError_t launch_probe_vectors(double* V, int64_t ldv, int64_t nGp, int64_t ng, int M, int d, hipStream_t st);
hipError_t launch_probe_band(double* ab, int64_t ldab, const double* Y, int64_t ldy, int64_t ng, int M, int d,
                             hipStream_t st);

}  // namespace td
