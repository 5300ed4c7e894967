// Frozen-step integration and its discrete adjoint (FP64, one thread per
// element).
//
// Forward: the Cash-Karp steps of section 2.2 on a given list of accepted
// steps (no error control), with the slip of eq. (16).  The arithmetic of a
// stage combination and of the update is that of the controlled integration,
// so a replay of its own step list reproduces it.
//
// Reverse (reverse-mode differentiation of those steps, per element; the
// transposed products are launched between the two halves of a stage):
//   slip term    D_{m+1} = D_m + dt/2 (V(y_m) + V(y_{m+1})): with Dbar the
//                cotangent of the final slip, dt/2 Dbar dV/dy goes to the
//                cotangents of y_m and y_{m+1}, dt/2 Dbar dV/da to abar;
//   stage s      kbar_s = dt b5_s ybar_{m+1} + dt sum_{r>s} a_rs Ybar_r,
//                Ybar_s = J_f(Y_s)^T kbar_s, f the right-hand side of
//                eqs. (8), (12), (13) (see k_vjp_pre / k_vjp_post);
//   state        ybar_m = ybar_{m+1} + sum_s Ybar_s.
// Parameters: a (with b fixed, so d/d(a - b) = d/da) and d_c, accumulated.
#include "device_types.hpp"
#include "rk_tableau.hpp"
#include "rs_adjoint.hpp"

namespace hm {
namespace {

constexpr int kBs = 256;

inline unsigned blocks(int64_t n) { return (unsigned)((n + kBs - 1) / kBs); }

__device__ __forceinline__ double slip_rate(double phi, double tau, double sig, double a, double V0) {
  const double q = tau / (a * sig), e = phi / a;
  return V0 * (exp(q - e) - exp(-q - e));
}

// y_out = y + dt sum_j b5_j k_j; D += dt/2 (V(y) + V(y_out)) (D may be null).
// y_out may alias y.
__global__ void k_update_dt(int64_t n, double dt, double V0, const double* __restrict__ a, const double* __restrict__ k,
                            const double* y, double* y_out, double* __restrict__ D) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t n3 = 3 * n;
  double v[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const int64_t e = c * n + i;
    double v5 = y[e];
    for (int j = 0; j < 6; ++j)
      if (kB5[j] != 0.0) v5 = v5 + (dt * kB5[j]) * k[j * n3 + e];
    v[c] = v5;
  }
  const double ai = a[i];
  if (D) {
    const double V = slip_rate(y[i], y[n + i], y[2 * n + i], ai, V0);
    const double V1 = slip_rate(v[0], v[1], v[2], ai, V0);
    D[i] = D[i] + 0.5 * dt * (V + V1);
  }
  y_out[i] = v[0];
  y_out[n + i] = v[1];
  y_out[2 * n + i] = v[2];
}

// slip term of one state: ybar += w Dbar dV/dy, abar += w Dbar dV/da, with
// V = V0 (ep - em), ep = exp(q - e), em = exp(-q - e), q = tau / (a sigma),
// e = phi / a.
__global__ void k_dterm(int64_t n, double w, double V0, const double* __restrict__ a, const double* __restrict__ y,
                        const double* __restrict__ Dbar, double* __restrict__ ybar, double* __restrict__ abar) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double phi = y[i], tau = y[n + i], sig = y[2 * n + i], ai = a[i];
  const double q = tau / (ai * sig), e = phi / ai;
  const double ep = exp(q - e), em = exp(-q - e);
  const double Vb = w * Dbar[i];
  const double qbar = V0 * Vb * (ep + em);
  const double ebar = -V0 * Vb * (ep - em);
  ybar[i] += ebar / ai;
  ybar[n + i] += qbar / (ai * sig);
  ybar[2 * n + i] += -(q / sig) * qbar;
  abar[i] += -(q / ai) * qbar - (e / ai) * ebar;
}

// First half of stage r: the stage cotangent kbar_r, and the cotangents of
// the two products of the right-hand side, gbar (of A x) and sbar (of B x).
// dtau/dt = num / den, num = A x - eta (V_s dsigma/dt + V_p dphi/dt),
// den = 1 + eta V_t (V_t, V_s, V_p: dV/dtau, dV/dsigma, dV/dphi), so
// gbar = kbar_tau / den, sbar = kbar_sigma - eta V_s gbar.
__global__ void k_vjp_pre(int64_t n, int r, double dt, double V0, double eta, const double* __restrict__ a,
                          const double* __restrict__ Y, const double* __restrict__ lam,
                          const double* __restrict__ Ybar, double* __restrict__ kbar, double* __restrict__ gbar,
                          double* __restrict__ sbar) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t n3 = 3 * n;
  double kb[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const int64_t e = c * n + i;
    double v = (dt * kB5[r]) * lam[e];
    for (int s = 5; s > r; --s) {
      const double cs = kA[s][r];
      if (cs != 0.0) v += (dt * cs) * Ybar[s * n3 + e];
    }
    kb[c] = v;
    kbar[e] = v;
  }
  const double tau = Y[n + i], sig = Y[2 * n + i], ai = a[i];
  const double q = tau / (ai * sig), e = Y[i] / ai;
  const double Vt = V0 / (ai * sig) * (exp(q - e) + exp(-q - e));
  const double Vs = -(tau / sig) * Vt;
  const double numbar = kb[1] / (1.0 + eta * Vt);
  gbar[i] = numbar;
  if (sbar) sbar[i] = kb[2] - eta * Vs * numbar;
}

// Second half of stage r: Ybar_r = J_f(Y_r)^T kbar_r given xa = A^T gbar and
// xb = B^T sbar (null: B = 0), and the cotangents of a and d_c.
//   dphi/dt = (b / d_c) (P - V), P = V0 exp((f0 - phi) / b)     (eq. (8))
//   V_t = C (ep + em), C = V0 / (a sigma); V_s = -(tau / sigma) V_t; V_p = -V / a
__global__ void k_vjp_post(int64_t n, double V0, double f0, double eta, const double* __restrict__ a,
                           const double* __restrict__ b, const double* __restrict__ dc, const double* __restrict__ Y,
                           const double* __restrict__ K, const double* __restrict__ kbar,
                           const double* __restrict__ xa, const double* __restrict__ xb, double* __restrict__ Ybar,
                           double* __restrict__ abar, double* __restrict__ dcbar) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double phi = Y[i], tau = Y[n + i], sig = Y[2 * n + i];
  const double ai = a[i], bi = b[i], dci = dc[i];
  const double dphi = K[i], dtau = K[n + i], dsig = K[2 * n + i];
  const double uphi = kbar[i], utau = kbar[n + i];
  // forward intermediates
  const double q = tau / (ai * sig), e = phi / ai;
  const double ep = exp(q - e), em = exp(-q - e);
  const double V = V0 * (ep - em);
  const double C = V0 / (ai * sig);
  const double Vt = C * (ep + em);
  const double Vp = -V / ai;
  const double den = 1.0 + eta * Vt;
  const double P = V0 * exp((f0 - phi) / bi);
  // eq. (12)
  const double numbar = utau / den;
  const double denbar = -utau * dtau / den;
  const double Vsbar = -eta * dsig * numbar;
  const double Vpbar = -eta * dphi * numbar;
  const double dphibar = uphi - eta * Vp * numbar;
  double Vtbar = eta * denbar;
  // eq. (8)
  const double Pbar = (bi / dci) * dphibar;
  double Vbar = -(bi / dci) * dphibar;
  const double dcb = -(dphi / dci) * dphibar;
  double phibar = -(P / bi) * Pbar;
  // V_p = -V / a
  Vbar -= Vpbar / ai;
  double ab = (V / (ai * ai)) * Vpbar;
  // V_s = -(tau / sigma) V_t
  double taubar = -(Vt / sig) * Vsbar;
  double sigbar = (tau * Vt / (sig * sig)) * Vsbar;
  Vtbar -= (tau / sig) * Vsbar;
  // the products: x = V - V_pl
  Vbar += xa[i];
  if (xb) Vbar += xb[i];
  // V_t = C (ep + em), V = V0 (ep - em)
  const double epbar = C * Vtbar + V0 * Vbar;
  const double embar = C * Vtbar - V0 * Vbar;
  const double Cbar = (ep + em) * Vtbar;
  ab -= (C / ai) * Cbar;
  sigbar -= (C / sig) * Cbar;
  // ep, em -> q, e -> tau, sigma, phi, a
  const double qbar = ep * epbar - em * embar;
  const double ebar = -ep * epbar - em * embar;
  taubar += qbar / (ai * sig);
  sigbar -= (q / sig) * qbar;
  ab -= (q / ai) * qbar;
  phibar += ebar / ai;
  ab -= (e / ai) * ebar;
  Ybar[i] = phibar;
  Ybar[n + i] = taubar;
  Ybar[2 * n + i] = sigbar;
  abar[i] += ab;
  dcbar[i] += dcb;
}

// ybar += Ybar_5 + Ybar_4 + ... + Ybar_0
__global__ void k_combine(int64_t n3, double* __restrict__ ybar, const double* __restrict__ Ybar) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n3) return;
  double v = ybar[i];
  for (int s = 5; s >= 0; --s) v += Ybar[s * n3 + i];
  ybar[i] = v;
}

}  // namespace

hipError_t launch_rk_update_dt(int64_t n, double dt, double V0, const double* a, const double* k, const double* y,
                               double* y_out, double* D, hipStream_t strm) {
  hipLaunchKernelGGL(k_update_dt, dim3(blocks(n)), dim3(kBs), 0, strm, n, dt, V0, a, k, y, y_out, D);
  return hipGetLastError();
}

hipError_t launch_adj_dterm(int64_t n, double w, double V0, const double* a, const double* y, const double* Dbar,
                            double* ybar, double* abar, hipStream_t strm) {
  hipLaunchKernelGGL(k_dterm, dim3(blocks(n)), dim3(kBs), 0, strm, n, w, V0, a, y, Dbar, ybar, abar);
  return hipGetLastError();
}

hipError_t launch_adj_vjp_pre(int64_t n, int r, double dt, const rs_params& p, const double* Y, const double* lam,
                              const double* Ybar, double* kbar, double* gbar, double* sbar, hipStream_t strm) {
  hipLaunchKernelGGL(k_vjp_pre, dim3(blocks(n)), dim3(kBs), 0, strm, n, r, dt, p.V0, p.eta_rad, p.a, Y, lam, Ybar,
                     kbar, gbar, sbar);
  return hipGetLastError();
}

hipError_t launch_adj_vjp_post(int64_t n, const rs_params& p, const double* Y, const double* K, const double* kbar,
                               const double* xa, const double* xb, double* Ybar, double* abar, double* dcbar,
                               hipStream_t strm) {
  hipLaunchKernelGGL(k_vjp_post, dim3(blocks(n)), dim3(kBs), 0, strm, n, p.V0, p.f0, p.eta_rad, p.a, p.b, p.dc, Y, K,
                     kbar, xa, xb, Ybar, abar, dcbar);
  return hipGetLastError();
}

hipError_t launch_adj_combine(int64_t n3, double* ybar, const double* Ybar, hipStream_t strm) {
  hipLaunchKernelGGL(k_combine, dim3(blocks(n3)), dim3(kBs), 0, strm, n3, ybar, Ybar);
  return hipGetLastError();
}

}  // namespace hm
