// Rate-and-state right-hand side kernels (section 2.2).
#pragma once

#include <hip/hip_runtime.h>

#include "device_types.hpp"
#include "rk_state.hpp"
#include "hmat.h"

namespace hm {

// V = 2 V0 exp(-phi/a) sinh(tau / (a sigma)) (eq. (7)); x = V - V_pl.
hipError_t launch_rs_slip_rate(int64_t n, double V0, double V_pl, const double* a, const double* y, double* x,
                               double* V_out, hipStream_t s);

// dy/dt from eqs. (8), (12), (13) given ax = A (V - V_pl) and bx = B (V - V_pl)
// (bx may be null: dsigma/dt = 0).
hipError_t launch_rs_rhs(int64_t n, const rs_params& p, const double* y, const double* ax, const double* bx,
                         double* dydt, hipStream_t s);

// One Runge-Kutta attempt is: launch_rk_begin, six stages (the slip rate of
// y for stage 0, launch_rk_stage_slip for stages 1..5; then the products and
// the right-hand side), then launch_rk_finish_control and launch_rk_accept.
// All read the step from the device state, so the sequence can be captured
// in a graph.
hipError_t launch_rk_begin(RkDevState* st, hipStream_t strm);
// Wall-clock stamp of a timed run (which: 0 attempt start, 1 product start,
// 2 product end, 3 attempt end).
hipError_t launch_rk_stamp(RkDevState* st, int which, hipStream_t strm);
// Cash-Karp stage input ys = y + dt sum_{j<s} a_sj k_j (k: 6 blocks of 3n,
// s in 1..5) and x = V(ys) - V_pl (eq. (7)).  dt is read from st, or taken
// from the argument when st is null (frozen steps).
hipError_t launch_rk_stage_slip(int64_t n, int s, const RkDevState* st, double dt, const double* y, const double* k,
                                double* ys, double V0, double V_pl, const double* a, double* x, hipStream_t strm);
// y5, the largest relative difference |y5 - y4| / |y5| and the step control.
hipError_t launch_rk_finish_control(int64_t n3, RkDevState* st, const double* y, const double* k, double* y5,
                                    hipStream_t strm);
// accepted step (if the controller accepted): eq. (16) slip update, y = y5;
// dt_log (or null) receives the step at index accepted - 1 - log_base.
hipError_t launch_rk_accept(int64_t n, const RkDevState* st, double V0, const double* a, const double* y5,
                            const double* Vstart, double* y, double* D, double* dt_log, hipStream_t strm);

}  // namespace hm
