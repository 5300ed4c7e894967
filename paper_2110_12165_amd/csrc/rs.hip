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

}  // namespace

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
