// Rate-and-state right-hand side kernels (section 2.2).
#pragma once

#include <hip/hip_runtime.h>

#include "hmat.h"

namespace hm {

// V = 2 V0 exp(-phi/a) sinh(tau / (a sigma)) (eq. (7)); x = V - V_pl.
hipError_t launch_rs_slip_rate(int64_t n, double V0, double V_pl, const double* a, const double* y, double* x,
                               double* V_out, hipStream_t s);

// dy/dt from eqs. (8), (12), (13) given ax = A (V - V_pl) and bx = B (V - V_pl)
// (bx may be null: dsigma/dt = 0).
hipError_t launch_rs_rhs(int64_t n, const rs_params& p, const double* y, const double* ax, const double* bx,
                         double* dydt, hipStream_t s);

}  // namespace hm
