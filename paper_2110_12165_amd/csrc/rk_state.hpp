// Runge-Kutta integration state shared by the host code and the kernels.
#pragma once

namespace hm {

// Slots of the error maximum: workgroup k of the error kernel folds its
// maximum into slot k % kErrSlots, so no single address takes every
// workgroup's atomic; the controller takes the maximum of the slots.
constexpr int kErrSlots = 8;

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
  unsigned long long err_bits[kErrSlots];  // max relative difference, as the bits of a non-negative double
  long long log_base;           // accepted count at which the step log starts
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
