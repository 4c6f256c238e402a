// Host-side declarations of the kernel launchers (one translation unit each).
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "common.h"

namespace hps {

// lu.hip: one kernel launch per schedule record (records of 8 ints, see common.h)
template <typename T>
hipError_t getrf_run(const Geom& g, const std::vector<int>& ops, T* A, int* perm, T* dinv, int* info, int nbox,
                     hipStream_t st);
template <typename T>
hipError_t getrs_run(const Geom& g, const std::vector<int>& fwd, const std::vector<int>& bwd, const T* F,
                     const int* perm, const T* dinv, const T* B, T* Y, int nbox, const int* active, hipStream_t st);

// leafops.hip
hipError_t launch_nodes(const Geom& g, const double* t, const double* h, int nbox, const double* origin, double* xi,
                        double* xb, hipStream_t st);
template <typename T>
hipError_t launch_operators(const Geom& g, int nbox, const double* b, T* A, double* anorm, hipStream_t st);
template <typename T>
hipError_t launch_rhs(const Geom& g, int nbox, const double* f, T* B, double* maxb, hipStream_t st);
hipError_t residual_prepare(const Geom& g);
hipError_t launch_residual(const Geom& g, int nbox, const double* b, const double* f, const double* X, float* R32,
                           double* maxr, double* maxx, const int* active, hipStream_t st);
hipError_t launch_ir_check(int nbox, int it, int last, double tol, const double* anorm, const double* maxb,
                           const double* maxr, const double* maxx, int* active, int* iters, double* berr,
                           hipStream_t st);
hipError_t launch_ir_add(const Geom& g, int nbox, const float* Y, double* X, int first, const int* active,
                         hipStream_t st);
hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t st);
hipError_t launch_fill_int(int* p, int value, size_t count, hipStream_t st);
hipError_t launch_dtn(const Geom& g, int nbox, const double* X, const double* gdir, const int* slot_map,
                      double* T_vals, double* gload, hipStream_t st);
hipError_t launch_reduce(int npairs, const long long* pairs, long long block_elems, double* T_vals, hipStream_t st);
hipError_t launch_reconstruct(const Geom& g, int nbox, const double* X, const double* ub, double* ui,
                              hipStream_t st);
hipError_t launch_adjoint_rhs(const Geom& g, int nbox, const double* w, const double* lam_b, double* rhs,
                              hipStream_t st);
hipError_t launch_getrs_t(const Geom& g, int nbox, const double* LU, const int* perm, const double* dinv,
                          const double* rhs, double* z, hipStream_t st);
hipError_t launch_adjoint_yb(const Geom& g, int nbox, const double* z, double* yb, hipStream_t st);
hipError_t launch_compact(const Geom& g, int nbox, const double* in, double* out, hipStream_t st);
hipError_t launch_grad(const Geom& g, int nbox, const double* lam, const double* u, double* grad, hipStream_t st);

}  // namespace hps
