// Ensemble integration kernels (section 2.2 per member): layout
// member-fastest, [(c n + i) M + r]; the per-member step and controller live
// in EnsDevState.  One attempt is: launch_ens_begin, six stages
// (launch_ens_slip for stage 0, launch_ens_stage_slip for stages 1..5; the
// ensemble products, launch_ens_rhs), launch_ens_finish_control,
// launch_ens_accept.
#pragma once

#include <algorithm>

#include <hip/hip_runtime.h>

#include "rk_state.hpp"

namespace hm {

hipError_t launch_ens_begin(EnsDevState* st, hipStream_t s);
// stage input ys = y + dt_r sum_{j<s} a_sj k_j (s in 1..5) and x = V(ys) - V_pl
hipError_t launch_ens_stage_slip(int64_t n, int M, int stage, const EnsDevState* st, const double* y, const double* k,
                                 double* ys, double V0, double V_pl, const double* a, double* x, hipStream_t s);
hipError_t launch_ens_slip(int64_t n, int M, double V0, double V_pl, const double* a, const double* y, double* x,
                           double* V_out, hipStream_t s);
hipError_t launch_ens_rhs(int64_t n, int M, double V0, double f0, double eta, const double* a, const double* b,
                          const double* dc, const double* y, const double* ax, const double* bx, double* dydt,
                          hipStream_t s);
hipError_t launch_ens_finish_control(int64_t n3, int M, EnsDevState* st, const double* y, const double* k, double* y5,
                                     hipStream_t s);
hipError_t launch_ens_accept(int64_t n, int M, const EnsDevState* st, double V0, const double* a, const double* y5,
                             const double* Vstart, double* y, double* D, hipStream_t s);

}  // namespace hm
