// Runge-Kutta integration state shared by the host code and the kernels.
#pragma once

namespace hm {

// Slots of the error maximum: workgroup k of the error kernel folds its
// maximum into slot k % kErrSlots, so no single address takes every
// workgroup's atomic; the controller takes the maximum of the slots.  Slot
// s is err_bits[s * kErrStride]: 128 bytes apart, each in a cache line of
// its own (atomics on one line are served one at a time).
constexpr int kErrSlots = 16;
constexpr int kErrStride = 16;
// Doubles at the end of the Runge-Kutta workspace that hold RkDevState.
constexpr int kRkStateDoubles = 288;

// Device-resident state of the adaptive Runge-Kutta integration: every
// kernel of an attempt reads the step from here, and the controller kernel
// (eqs. (14)-(15)) updates it, so attempts can be replayed from a graph with
// no host round trip.
struct RkDevState {
  double t, dt, eps, r, dt_used;
  long long accepted, rejected, target;
  int force;        // -1 controller decides, 0 reject, 1 accept
  int ok;           // decision of the last attempt
  int halted;       // target reached: further attempts change nothing
  int pad;
  long long log_base;           // accepted count at which the step log starts
  // wall-clock stamps of a timed run (rs_rk45_run_timed): start of the
  // attempt and of the current product pair, and the summed ticks of the
  // product pairs and of the attempts
  unsigned long long prof_a0, prof_t0, prof_prod, prof_att;
  unsigned long long err_bits[kErrSlots * kErrStride];  // max relative difference, as the bits of a
                                                        // non-negative double (slots as above)
};

}  // namespace hm

namespace hm {

// Device-resident state of an ensemble integration: up to 64 members, each
// with its own step, controller decision and counters (the members share the
// products, not the steps).
constexpr int kEnsMax = 64;
struct EnsDevState {
  double t[kEnsMax], dt[kEnsMax], dt_used[kEnsMax], r[kEnsMax];
  unsigned long long err_bits[kEnsMax];  // per-member max relative difference (bits of a double)
  long long accepted[kEnsMax], rejected[kEnsMax], target[kEnsMax];
  int ok[kEnsMax], halted[kEnsMax];
  double eps;
  int members, pad;
};

}  // namespace hm
