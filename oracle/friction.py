"""Rate-and-state right-hand side (FP64, NumPy).

Paper: section 2.2, eqs. (7)-(13); loading of section 4.1, eqs. (21)-(22).

Reading of eq. (7): printed as tau/sigma = a asinh(V/(2 V0) exp(-phi)), which
does not agree with eqs. (8) and (13c).  Read with the state entering as
exp(-phi/a) (the regularised law used with the aging law of eq. 8):

    V = 2 V0 exp(-phi/a) sinh(tau / (a sigma)),
    tau = a sigma asinh( V / (2 V0) * exp(phi/a) ),

so that at steady state (eq. 8: V0 exp((f0 - phi)/b) = V) the friction is
f0 + (a - b) ln(V/V0) for large V/V0.  Eqs. (13a-c) are the partial
derivatives of this V (with exp(-phi/a)); eq. (12) uses S = A.

State vector y = (phi_1..N, tau_1..N, sigma_1..N).  The backslip loading
tau_dot = -V_pl sum_j A_ij (eq. 21) and sigma_dot = -V_pl sum_j B_ij (eq. 22)
are applied by multiplying A and B with V - V_pl.

Pins (tests/test_oracle_friction.py): round trip V(tau(V)) = V; the partial
derivatives against complex-step derivatives; the steady-state friction
against f0 + (a-b) ln(V/V0); the plate-rate fixed point dy/dt = 0; the
radiation-damping elimination of eq. (11) checked by finite differences of
a quasi-dynamic force balance; the state rate of eq. (8) away from steady
state against the theta form of the aging law (dtheta/dt = 1 - V theta/d_c);
the critical stiffness of a one-element spring-slider, where the linearised
right-hand side loses stability, against sigma (b - a) / d_c (less the
radiation-damping shift eta V_pl / d_c).
"""
from __future__ import annotations

import numpy as np


def slip_rate(phi, tau, sigma, a, V0):
    """Eq. (7) solved for V (works for complex arguments, for complex-step tests)."""
    q = tau / (a * sigma)
    e = phi / a
    return V0 * (np.exp(q - e) - np.exp(-q - e))


def shear_traction(V, phi, sigma, a, V0):
    """Eq. (7): tau = a sigma asinh(V / (2 V0) exp(phi / a))."""
    return a * sigma * np.arcsinh(V / (2.0 * V0) * np.exp(phi / a))


def steady_state_phi(V, b, V0, f0):
    """Eq. (8) with dphi/dt = 0: phi = f0 + b ln(V0 / V)."""
    return f0 + b * np.log(V0 / V)


def partials(phi, tau, sigma, a, V0):
    """Eqs. (13a-c): dV/dtau, dV/dsigma, dV/dphi."""
    q = tau / (a * sigma)
    e = phi / a
    dV_dtau = V0 / (a * sigma) * (np.exp(q - e) + np.exp(-q - e))
    dV_dsigma = -(tau / sigma) * dV_dtau
    dV_dphi = -slip_rate(phi, tau, sigma, a, V0) / a
    return dV_dtau, dV_dsigma, dV_dphi


def rhs(y, p, apply_A, apply_B=None):
    """dy/dt (eqs. 8, 10, 12).  p: dict with a, b, dc (arrays), V0, f0,
    eta_rad, V_pl.  apply_A(x) -> A x (user order); apply_B likewise or None
    (B = 0).  Returns (dydt, V)."""
    n = y.shape[0] // 3
    phi, tau, sig = y[:n], y[n:2 * n], y[2 * n:]
    a, b, dc = p["a"], p["b"], p["dc"]
    V = slip_rate(phi, tau, sig, a, p["V0"])
    x = V - p["V_pl"]
    ax = apply_A(x)
    dsig = apply_B(x) if apply_B is not None else np.zeros(n)
    dphi = b / dc * (p["V0"] * np.exp((p["f0"] - phi) / b) - V)          # eq. (8)
    dV_dtau, dV_dsig, dV_dphi = partials(phi, tau, sig, a, p["V0"])      # eq. (13)
    eta = p["eta_rad"]
    dtau = (ax - eta * (dV_dsig * dsig + dV_dphi * dphi)) / (1.0 + eta * dV_dtau)   # eq. (12)
    return np.concatenate([dphi, dtau, dsig]), V


def initial_state(V_init, p, sigma):
    """Steady state at slip rate V_init: phi = phi_ss(V_init), tau from eq. (7)."""
    V_init = np.broadcast_to(np.asarray(V_init, dtype=np.float64), sigma.shape)
    phi = steady_state_phi(V_init, p["b"], p["V0"], p["f0"])
    tau = shear_traction(V_init, phi, sigma, p["a"], p["V0"])
    return np.concatenate([phi, tau, np.asarray(sigma, dtype=np.float64)])
