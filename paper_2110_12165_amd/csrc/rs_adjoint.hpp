// Frozen-step Runge-Kutta integration and its discrete adjoint (section 2.2
// integrator differentiated in reverse mode).  All FP64, element-wise; the
// products with A, B, A^T and B^T are launched by the caller between them.
#pragma once

#include <hip/hip_runtime.h>

#include "hmat.h"

namespace hm {

// y_out = y + dt sum_j b5_j k_j and D += dt/2 (V(y) + V(y_out)) (eq. (16);
// D may be null); y_out may alias y.
hipError_t launch_rk_update_dt(int64_t n, double dt, double V0, const double* a, const double* k, const double* y,
                               double* y_out, double* D, hipStream_t strm);
// ybar += w Dbar dV/dy and abar += w Dbar dV/da at state y.
hipError_t launch_adj_dterm(int64_t n, double w, double V0, const double* a, const double* y, const double* Dbar,
                            double* ybar, double* abar, hipStream_t strm);
// Stage r, first half: kbar_r = dt b5_r lam + dt sum_{s>r} a_sr Ybar_s (Ybar:
// 6 blocks of 3n), gbar = cotangent of A x, sbar = cotangent of B x (sbar may
// be null when B = 0).  Y: the stage input (3n).
hipError_t launch_adj_vjp_pre(int64_t n, int r, double dt, const rs_params& p, const double* Y, const double* lam,
                              const double* Ybar, double* kbar, double* gbar, double* sbar, hipStream_t strm);
// Stage r, second half: Ybar_r (3n) from xa = A^T gbar and xb = B^T sbar
// (null when B = 0); abar and dcbar accumulate.  K: the stage derivative (3n).
hipError_t launch_adj_vjp_post(int64_t n, const rs_params& p, const double* Y, const double* K, const double* kbar,
                               const double* xa, const double* xb, double* Ybar, double* abar, double* dcbar,
                               hipStream_t strm);
// ybar += sum_s Ybar_s.
hipError_t launch_adj_combine(int64_t n3, double* ybar, const double* Ybar, hipStream_t strm);

}  // namespace hm
