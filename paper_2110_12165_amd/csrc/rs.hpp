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

// Cash-Karp stage input ys = y + dt sum_{j<s} a_sj k_j (k: 6 blocks of n3).
hipError_t launch_rk_stage(int64_t n3, int s, double dt, const double* y, const double* k, double* ys,
                           hipStream_t st);
// y5 and the largest relative difference |y5 - y4| / |y5| (bits of a
// non-negative double, atomic max; cleared by the launch itself).
hipError_t launch_rk_finish(int64_t n3, double dt, const double* y, const double* k, double* y5,
                            unsigned long long* err_bits, hipStream_t st);
// accepted step: slip update of eq. (16) and y = y5.
hipError_t launch_rk_accept(int64_t n, double dt, double V0, const double* a, const double* y5, const double* Vstart,
                            double* y, double* D, hipStream_t st);

}  // namespace hm
