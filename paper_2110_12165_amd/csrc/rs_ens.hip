// Ensemble integration: up to 64 rate-and-state simulations on one fault,
// advanced together (section 2.2, eqs. (7)-(16) per member).  Every member
// has its own parameters (a, b, d_c per element), state, slip, step and step
// control; at every Runge-Kutta stage the slip-rate block of all members
// goes through one ensemble product with A (and B).  All element-wise work
// is FP64.
//
// Layout: member-fastest, y[(c n + i) M + r] for component c (phi, tau,
// sigma), element i, member r (M members), matching the ensemble product's
// X[i ldx + r]; parameters and slip as [i M + r].  Threads: blockDim = (64, 4),
// x = member, y = element lane.
#include "device_types.hpp"
#include "rk_state.hpp"
#include "rk_tableau.hpp"
#include "rs_ens.hpp"

namespace hm {
namespace {

__device__ __forceinline__ double slip_rate(double phi, double tau, double sig, double a, double V0) {
  const double q = tau / (a * sig), e = phi / a;
  return V0 * (exp(q - e) - exp(-q - e));
}

// elements e (of n_el) handled by this thread, member r; false when idle
__device__ __forceinline__ bool elem(int64_t n_el, int M, int64_t& e, int& r) {
  r = threadIdx.x;
  e = (int64_t)blockIdx.x * blockDim.y + threadIdx.y;
  return r < M && e < n_el;
}

__global__ void k_ens_begin(EnsDevState* st) {
  if (threadIdx.x < kEnsMax) st->err_bits[threadIdx.x] = 0ull;
}

// Stage input ys = y + dt_r sum_{j<s} a_sj k_j (the three components of
// element i, member r) and the product input x = V(ys) - V_pl, in one pass.
__global__ void k_ens_stage_slip(int64_t n, int M, int s, const EnsDevState* __restrict__ st,
                                 const double* __restrict__ y, const double* __restrict__ k, double* __restrict__ ys,
                                 double V0, double V_pl, const double* __restrict__ a, double* __restrict__ x) {
  int64_t i;
  int r;
  if (!elem(n, M, i, r)) return;
  const int64_t nm = n * M, stride = 3 * nm;
  const double dt = st->dt[r];
  double v[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const int64_t idx = c * nm + i * M + r;
    double w = y[idx];
    for (int j = 0; j < s; ++j) {
      const double cf = kA[s][j];
      if (cf != 0.0) w = w + (dt * cf) * k[j * stride + idx];
    }
    ys[idx] = w;
    v[c] = w;
  }
  x[i * M + r] = slip_rate(v[0], v[1], v[2], a[i * M + r], V0) - V_pl;
}

// x = V(y) - V_pl (eq. (7)); V_out (or null) receives V
__global__ void k_ens_slip(int64_t n, int M, double V0, double V_pl, const double* __restrict__ a,
                           const double* __restrict__ y, double* __restrict__ x, double* __restrict__ V_out) {
  int64_t i;
  int r;
  if (!elem(n, M, i, r)) return;
  const int64_t idx = i * M + r, nm = n * M;
  const double V = slip_rate(y[idx], y[nm + idx], y[2 * nm + idx], a[idx], V0);
  x[idx] = V - V_pl;
  if (V_out) V_out[idx] = V;
}

// dy/dt (eqs. (8), (12), (13)) from ax = A x and bx = B x (bx may be null)
__global__ void k_ens_rhs(int64_t n, int M, double V0, double f0, double eta, const double* __restrict__ a,
                          const double* __restrict__ b, const double* __restrict__ dc, const double* __restrict__ y,
                          const double* __restrict__ ax, const double* __restrict__ bx, double* __restrict__ dydt) {
  int64_t i;
  int r;
  if (!elem(n, M, i, r)) return;
  const int64_t idx = i * M + r, nm = n * M;
  const double phi = y[idx], tau = y[nm + idx], sig = y[2 * nm + idx];
  const double ai = a[idx], bi = b[idx];
  const double q = tau / (ai * sig), e = phi / ai;
  const double ep = exp(q - e), em = exp(-q - e);
  const double V = V0 * (ep - em);
  const double dV_dtau = V0 / (ai * sig) * (ep + em);
  const double dV_dsig = -(tau / sig) * dV_dtau;
  const double dV_dphi = -V / ai;
  const double dphi = bi / dc[idx] * (V0 * exp((f0 - phi) / bi) - V);
  const double dsig = bx ? bx[idx] : 0.0;
  dydt[idx] = dphi;
  dydt[nm + idx] = (ax[idx] - eta * (dV_dsig * dsig + dV_dphi * dphi)) / (1.0 + eta * dV_dtau);
  dydt[2 * nm + idx] = dsig;
}

// y5 and, per member, max |y5 - y4| / max(|y5|, 1e-300) over its 3n unknowns
// (NaN wins).  Elements are strided over the grid; the four element lanes of
// a block are combined in LDS, then one atomic max per member and block.
__global__ __launch_bounds__(256) void k_ens_finish(int64_t n3, int M, EnsDevState* st, const double* __restrict__ y,
                                                    const double* __restrict__ k, double* __restrict__ y5) {
  __shared__ double part[4][kEnsMax];
  const int r = threadIdx.x;
  const int64_t stride = n3 * M;
  double m = 0.0;
  if (r < M) {
    const double dt = st->dt[r];
    for (int64_t e = (int64_t)blockIdx.x * blockDim.y + threadIdx.y; e < n3; e += (int64_t)gridDim.x * blockDim.y) {
      const int64_t idx = e * M + r;
      double v5 = y[idx], v4 = y[idx];
      for (int j = 0; j < 6; ++j) {
        const double kj = k[j * stride + idx];
        if (kB5[j] != 0.0) v5 = v5 + (dt * kB5[j]) * kj;
        if (kB4[j] != 0.0) v4 = v4 + (dt * kB4[j]) * kj;
      }
      y5[idx] = v5;
      double d = fabs(v5 - v4) / fmax(fabs(v5), 1e-300);
      if (d != d) d = __longlong_as_double(0x7ff8000000000000ll);
      m = (d != d || d > m) ? d : m;
    }
  }
  part[threadIdx.y][r] = m;
  __syncthreads();
  if (threadIdx.y == 0 && r < M) {
    for (int w = 1; w < (int)blockDim.y; ++w) m = (part[w][r] != part[w][r] || part[w][r] > m) ? part[w][r] : m;
    atomicMax(&st->err_bits[r], (unsigned long long)__double_as_longlong(m));
  }
}

// Step control per member (eqs. (14)-(15)), as for a single simulation.
__global__ void k_ens_control(EnsDevState* st) {
  const int r = threadIdx.x;
  if (r >= st->members) return;
  if (st->halted[r]) {
    st->ok[r] = 0;
    return;
  }
  const double err = __longlong_as_double((long long)st->err_bits[r]);
  const double q = err / st->eps;
  const double dt = st->dt[r];
  const bool finite = q == q && q != __longlong_as_double(0x7ff0000000000000ll);
  const bool ok = finite && q <= 1.0;
  st->r[r] = q;
  st->ok[r] = ok ? 1 : 0;
  st->dt_used[r] = dt;
  if (ok) {
    st->t[r] = st->t[r] + dt;
    st->accepted[r] += 1;
  } else {
    st->rejected[r] += 1;
  }
  if (!finite) st->dt[r] = 0.5 * dt;
  else if (ok) st->dt[r] = q == 0.0 ? 2.0 * dt : fmin(2.0 * dt, 0.9 * dt * pow(q, -0.2));
  else st->dt[r] = fmax(0.5 * dt, 0.9 * dt * pow(q, -0.25));
  if (st->accepted[r] >= st->target[r]) st->halted[r] = 1;
}

// accepted members: D += dt/2 (V(y) + V(y5)) (eq. (16)); y = y5
__global__ void k_ens_accept(int64_t n, int M, const EnsDevState* __restrict__ st, double V0,
                             const double* __restrict__ a, const double* __restrict__ y5,
                             const double* __restrict__ Vstart, double* __restrict__ y, double* __restrict__ D) {
  int64_t i;
  int r;
  if (!elem(n, M, i, r) || !st->ok[r]) return;
  const int64_t idx = i * M + r, nm = n * M;
  const double dt = st->dt_used[r];
  const double phi = y5[idx], tau = y5[nm + idx], sig = y5[2 * nm + idx];
  const double V1 = slip_rate(phi, tau, sig, a[idx], V0);
  D[idx] = D[idx] + 0.5 * dt * (Vstart[idx] + V1);
  y[idx] = phi;
  y[nm + idx] = tau;
  y[2 * nm + idx] = sig;
}

inline dim3 grid_for(int64_t n_el) { return dim3((unsigned)((n_el + 3) / 4)); }

}  // namespace

hipError_t launch_ens_begin(EnsDevState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_ens_begin, dim3(1), dim3(kEnsMax), 0, s, st);
  return hipGetLastError();
}

hipError_t launch_ens_stage_slip(int64_t n, int M, int stage, const EnsDevState* st, const double* y, const double* k,
                                 double* ys, double V0, double V_pl, const double* a, double* x, hipStream_t s) {
  if (stage < 1 || stage > 5) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_ens_stage_slip, grid_for(n), dim3(kEnsMax, 4), 0, s, n, M, stage, st, y, k, ys, V0, V_pl, a,
                     x);
  return hipGetLastError();
}

hipError_t launch_ens_slip(int64_t n, int M, double V0, double V_pl, const double* a, const double* y, double* x,
                           double* V_out, hipStream_t s) {
  hipLaunchKernelGGL(k_ens_slip, grid_for(n), dim3(kEnsMax, 4), 0, s, n, M, V0, V_pl, a, y, x, V_out);
  return hipGetLastError();
}

hipError_t launch_ens_rhs(int64_t n, int M, double V0, double f0, double eta, const double* a, const double* b,
                          const double* dc, const double* y, const double* ax, const double* bx, double* dydt,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_ens_rhs, grid_for(n), dim3(kEnsMax, 4), 0, s, n, M, V0, f0, eta, a, b, dc, y, ax, bx, dydt);
  return hipGetLastError();
}

hipError_t launch_ens_finish_control(int64_t n3, int M, EnsDevState* st, const double* y, const double* k, double* y5,
                                     hipStream_t s) {
  const unsigned blocks = (unsigned)std::min<int64_t>((n3 + 3) / 4, 2048);
  hipLaunchKernelGGL(k_ens_finish, dim3(blocks), dim3(kEnsMax, 4), 0, s, n3, M, st, y, k, y5);
  hipLaunchKernelGGL(k_ens_control, dim3(1), dim3(kEnsMax), 0, s, st);
  return hipGetLastError();
}

hipError_t launch_ens_accept(int64_t n, int M, const EnsDevState* st, double V0, const double* a, const double* y5,
                             const double* Vstart, double* y, double* D, hipStream_t s) {
  hipLaunchKernelGGL(k_ens_accept, grid_for(n), dim3(kEnsMax, 4), 0, s, n, M, st, V0, a, y5, Vstart, y, D);
  return hipGetLastError();
}

}  // namespace hm
