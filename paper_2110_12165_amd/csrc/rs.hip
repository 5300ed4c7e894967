// Rate-and-state right-hand side (section 2.2, eqs. (7)-(13); loading of
// section 4.1, eqs. (21)-(22)), FP64, one thread per element.
//
// Regularised friction law, read with the state entering as exp(-phi/a):
//   V = 2 V0 exp(-phi/a) sinh(tau / (a sigma))
// evaluated as V0 [exp(q - phi/a) - exp(-q - phi/a)], q = tau / (a sigma),
// which cannot overflow for physical states.  Its partial derivatives:
//   dV/dtau   = V0 / (a sigma) [exp(q - phi/a) + exp(-q - phi/a)]
//   dV/dsigma = -(tau / sigma) dV/dtau
//   dV/dphi   = -V / a
// Aging law:        dphi/dt = (b / d_c) [V0 exp((f0 - phi) / b) - V]
// Normal stress:    dsigma/dt = (B (V - V_pl))_i
// Shear stress with radiation damping eta = mu / (2 c_s), dV/dt eliminated:
//   dtau/dt = [ (A (V - V_pl))_i - eta (dV/dsigma dsigma/dt + dV/dphi dphi/dt) ]
//             / (1 + eta dV/dtau)
// The backslip loading tau_dot = -V_pl sum_j A_ij is folded into the product
// by applying A to V - V_pl.
#include <algorithm>

#include "device_types.hpp"
#include "rk_state.hpp"
#include "rk_tableau.hpp"
#include "rs.hpp"

namespace hm {
namespace {

__global__ void k_slip_rate(int64_t n, double V0, double V_pl, const double* __restrict__ a,
                            const double* __restrict__ y, double* __restrict__ x, double* __restrict__ V_out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double phi = y[i], tau = y[n + i], sig = y[2 * n + i];
  const double ai = a[i];
  const double q = tau / (ai * sig);
  const double e = phi / ai;
  const double V = V0 * (exp(q - e) - exp(-q - e));
  x[i] = V - V_pl;
  if (V_out) V_out[i] = V;
}

__global__ void k_rhs(int64_t n, double V0, double f0, double eta, const double* __restrict__ a,
                      const double* __restrict__ b, const double* __restrict__ dc, const double* __restrict__ y,
                      const double* __restrict__ ax, const double* __restrict__ bx, double* __restrict__ dydt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double phi = y[i], tau = y[n + i], sig = y[2 * n + i];
  const double ai = a[i], bi = b[i];
  const double q = tau / (ai * sig);
  const double e = phi / ai;
  const double ep = exp(q - e), em = exp(-q - e);
  const double V = V0 * (ep - em);
  const double dV_dtau = V0 / (ai * sig) * (ep + em);
  const double dV_dsig = -(tau / sig) * dV_dtau;
  const double dV_dphi = -V / ai;
  const double dphi = bi / dc[i] * (V0 * exp((f0 - phi) / bi) - V);
  const double dsig = bx ? bx[i] : 0.0;
  const double dtau = (ax[i] - eta * (dV_dsig * dsig + dV_dphi * dphi)) / (1.0 + eta * dV_dtau);
  dydt[i] = dphi;
  dydt[n + i] = dtau;
  dydt[2 * n + i] = dsig;
}

// ---------------------------------------------------------------------------
// Embedded Runge-Kutta 5(4) of Cash & Karp (1990): stage combinations, the
// relative difference of the two solutions (section 2.2) and the accepted
// update with the trapezoidal slip rule of eq. (16).
// ---------------------------------------------------------------------------
// Stage input ys = y + dt * sum_{j<s} a_sj k_j (the three components of
// element i) and the product input x_i = V(ys_i) - V_pl, in one pass.  The
// step comes from the device state st or, when st is null, from dt.
__global__ void k_stage_slip(int64_t n, int s, const RkDevState* __restrict__ st, double dt_val,
                             const double* __restrict__ y, const double* __restrict__ k, double* __restrict__ ys,
                             double V0, double V_pl, const double* __restrict__ a, double* __restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t n3 = 3 * n;
  const double dt = st ? st->dt : dt_val;
  double v[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const int64_t e = c * n + i;
    double w = y[e];
    for (int j = 0; j < s; ++j) {
      const double cf = kA[s][j];
      if (cf != 0.0) w = w + (dt * cf) * k[j * n3 + e];
    }
    ys[e] = w;
    v[c] = w;
  }
  const double ai = a[i];
  const double q = v[1] / (ai * v[2]);
  const double ee = v[0] / ai;
  const double V = V0 * (exp(q - ee) - exp(-q - ee));
  x[i] = V - V_pl;
}

// Wall-clock stamps of a timed run (one thread): 0 starts an attempt, 1 a
// product pair, 2 ends the pair (its ticks summed), 3 ends the attempt.
__global__ void k_stamp(RkDevState* st, int which) {
  const unsigned long long now = wall_clock64();
  switch (which) {
    case 0: st->prof_a0 = now; break;
    case 1: st->prof_t0 = now; break;
    case 2: st->prof_prod += now - st->prof_t0; break;
    default: st->prof_att += now - st->prof_a0; break;
  }
}

__global__ void k_begin(RkDevState* st) {
  if (threadIdx.x < kErrSlots) st->err_bits[threadIdx.x * kErrStride] = 0ull;
}

// y5, and max_i |y5 - y4| / max(|y5|, 1e-300) (non-negative doubles order like
// their bit patterns, so the maximum is an integer atomic max; NaN wins).
// Grid-stride over the 3n components with at most kFinishBlocks workgroups
// (one component per thread up to n3 = 2^20); k_1 has weight 0 in both
// solutions of the pair and is not read.  Each workgroup folds its maximum
// into one of the kErrSlots slots: the result does not depend on the grid
// (a maximum is exact in any order).
constexpr int kFinishThreads = 256;
constexpr int kFinishBlocks = 4096;

__global__ __launch_bounds__(kFinishThreads) void k_finish(int64_t n3, RkDevState* st, const double* __restrict__ y,
                                                           const double* __restrict__ k, double* __restrict__ y5) {
  __shared__ double part[kFinishThreads / 64];
  const double dt = st->dt;
  double c5[6], c4[6];
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    c5[j] = dt * kB5[j];
    c4[j] = dt * kB4[j];
  }
  double e = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kFinishThreads + threadIdx.x; i < n3;
       i += (int64_t)gridDim.x * kFinishThreads) {
    double v5 = y[i], v4 = v5;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      if (kB5[j] == 0.0 && kB4[j] == 0.0) continue;
      const double kj = k[j * n3 + i];
      if (kB5[j] != 0.0) v5 = v5 + c5[j] * kj;
      if (kB4[j] != 0.0) v4 = v4 + c4[j] * kj;
    }
    y5[i] = v5;
    double ei = fabs(v5 - v4) / fmax(fabs(v5), 1e-300);
    if (ei != ei) ei = __longlong_as_double(0x7ff8000000000000ll);
    e = (ei != ei || ei > e) ? ei : e;
  }
  for (int d = 32; d >= 1; d >>= 1) {
    const double o = __shfl_xor(e, d, 64);
    e = (o != o || o > e) ? o : e;
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) part[wave] = e;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = part[0];
    for (int w = 1; w < kFinishThreads / 64; ++w) m = (part[w] != part[w] || part[w] > m) ? part[w] : m;
    atomicMax(&st->err_bits[(blockIdx.x % kErrSlots) * kErrStride], (unsigned long long)__double_as_longlong(m));
  }
}

// Step control, one thread: accept if r = err / eps_RK <= 1 (finite), then
//   accept: dt <- min(2 dt, 0.9 dt r^(-1/5))  (2 dt if r = 0)     eq. (15)
//   reject: dt <- max(dt / 2, 0.9 dt r^(-1/4))                    eq. (14)
// non-finite r: reject, dt / 2.  A forced decision leaves dt unchanged.
__global__ void k_control(RkDevState* st) {
  if (st->halted) {
    st->ok = 0;
    return;
  }
  unsigned long long bits = st->err_bits[0];
  for (int q = 1; q < kErrSlots; ++q) {
    const unsigned long long v = st->err_bits[q * kErrStride];
    bits = v > bits ? v : bits;
  }
  const double err = __longlong_as_double((long long)bits);
  const double r = err / st->eps;
  const double dt = st->dt;
  const bool finite = r == r && r != __longlong_as_double(0x7ff0000000000000ll);
  const bool ok = st->force >= 0 ? st->force == 1 : (finite && r <= 1.0);
  st->r = r;
  st->ok = ok ? 1 : 0;
  st->dt_used = dt;
  if (ok) {
    st->t = st->t + dt;
    st->accepted += 1;
  } else {
    st->rejected += 1;
  }
  if (st->force < 0) {
    if (!finite) st->dt = 0.5 * dt;
    else if (ok) st->dt = r == 0.0 ? 2.0 * dt : fmin(2.0 * dt, 0.9 * dt * pow(r, -0.2));
    else st->dt = fmax(0.5 * dt, 0.9 * dt * pow(r, -0.25));
  }
  if (st->accepted >= st->target) st->halted = 1;
}

// accepted step: D += dt/2 (V(y) + V(y5)) (eq. 16); y = y5
__global__ void k_accept(int64_t n, const RkDevState* __restrict__ st, double V0, const double* __restrict__ a,
                         const double* __restrict__ y5, const double* __restrict__ Vstart, double* __restrict__ y,
                         double* __restrict__ D, double* __restrict__ dt_log) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || !st->ok) return;
  const double dt = st->dt_used;
  if (dt_log && i == 0) dt_log[st->accepted - 1 - st->log_base] = dt;
  const double phi = y5[i], tau = y5[n + i], sig = y5[2 * n + i];
  const double ai = a[i];
  const double q = tau / (ai * sig), e = phi / ai;
  const double V1 = V0 * (exp(q - e) - exp(-q - e));
  D[i] = D[i] + 0.5 * dt * (Vstart[i] + V1);
  y[i] = phi;
  y[n + i] = tau;
  y[2 * n + i] = sig;
}

}  // namespace

hipError_t launch_rk_stage_slip(int64_t n, int s, const RkDevState* st, double dt, const double* y, const double* k,
                                double* ys, double V0, double V_pl, const double* a, double* x, hipStream_t strm) {
  if (s < 1 || s > 5) return hipErrorInvalidValue;
  const int bs = 256;
  hipLaunchKernelGGL(k_stage_slip, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, strm, n, s, st, dt, y, k, ys, V0,
                     V_pl, a, x);
  return hipGetLastError();
}

hipError_t launch_rk_stamp(RkDevState* st, int which, hipStream_t strm) {
  hipLaunchKernelGGL(k_stamp, dim3(1), dim3(1), 0, strm, st, which);
  return hipGetLastError();
}

hipError_t launch_rk_begin(RkDevState* st, hipStream_t strm) {
  hipLaunchKernelGGL(k_begin, dim3(1), dim3(64), 0, strm, st);
  return hipGetLastError();
}

hipError_t launch_rk_finish_control(int64_t n3, RkDevState* st, const double* y, const double* k, double* y5,
                                    hipStream_t strm) {
  const int64_t blocks = std::min<int64_t>(kFinishBlocks, (n3 + kFinishThreads - 1) / kFinishThreads);
  hipLaunchKernelGGL(k_finish, dim3((unsigned)std::max<int64_t>(1, blocks)), dim3(kFinishThreads), 0, strm, n3, st, y,
                     k, y5);
  hipLaunchKernelGGL(k_control, dim3(1), dim3(1), 0, strm, st);
  return hipGetLastError();
}

hipError_t launch_rk_accept(int64_t n, const RkDevState* st, double V0, const double* a, const double* y5,
                            const double* Vstart, double* y, double* D, double* dt_log, hipStream_t strm) {
  const int bs = 256;
  hipLaunchKernelGGL(k_accept, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, strm, n, st, V0, a, y5, Vstart, y,
                     D, dt_log);
  return hipGetLastError();
}

hipError_t launch_rs_slip_rate(int64_t n, double V0, double V_pl, const double* a, const double* y, double* x,
                               double* V_out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int bs = 256;
  hipLaunchKernelGGL(k_slip_rate, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, s, n, V0, V_pl, a, y, x, V_out);
  return hipGetLastError();
}

hipError_t launch_rs_rhs(int64_t n, const rs_params& p, const double* y, const double* ax, const double* bx,
                         double* dydt, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int bs = 256;
  hipLaunchKernelGGL(k_rhs, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, s, n, p.V0, p.f0, p.eta_rad, p.a, p.b,
                     p.dc, y, ax, bx, dydt);
  return hipGetLastError();
}

}  // namespace hm
