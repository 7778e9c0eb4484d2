// host_common.hpp -- host-side helpers shared by the library's entry points.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "automat.h"
#include "msgsm.hpp"

namespace automat {

// Validate an automat_params table and convert it to the kernels' layout.
int32_t copy_params(const automat_params *params, MSGSM::Phase *dst, int32_t *n_phases);

// One evaluation sweep that writes the polarization tau = sigma - C0 eps
// (isotropic C0 = (lam0, mu0)) instead of sigma, for the basic scheme; no
// a_{n+1}, tangent or iteration output. The Newton solves start from the
// increments in delta [6][n] (device, or null for zero), which receive the
// converged increments. nonconverged (device, or null) counts the point
// solves that failed.
int32_t evaluate_polarized(int64_t n, const double *eps, const double *a_old,
                           const uint8_t *phase, const automat_params *params, double h,
                           double tol, int32_t max_iter, double lam0, double mu0, double *tau_out,
                           double *delta, uint64_t *nonconverged, void *stream);

// Evaluation whose Newton solves start from guess [6][n] (device, or null
// for zero) instead of a zero increment; delta_out [6][n] (or null, may
// equal guess) receives the converged increments a_{n+1} - a_n.
int32_t evaluate_warm(int64_t n, const double *eps, const double *a_old, const uint8_t *phase,
                      const automat_params *params, double h, double tol, int32_t max_iter,
                      double *sigma_out, double *a_out, double *tangent_out, const double *guess,
                      double *delta_out, uint64_t *nonconverged, void *stream);

// Compute-unit count of the current device (cached per device).
int32_t device_cus(int *cus);

}  // namespace automat
