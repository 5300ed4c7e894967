"""Discrete adjoint of the rate-and-state integration on a frozen step
sequence (FP64, NumPy).  Test infrastructure, like the rest of this package.

What is differentiated.  The forward map is the integration of section 2.2
(right-hand side of eqs. (7)-(13) with the loading of eqs. (21)-(22),
Cash-Karp steps, slip by the trapezoidal rule of eq. (16)) replayed on a
fixed list of accepted steps dt_0 .. dt_{M-1}: the error control of
eqs. (14)-(15) only chose those steps, so with the list frozen every step is
a smooth function of the state and the parameters.  The parameters are the
per-element a (b held fixed, so a derivative with respect to a - b is one
with respect to a) and d_c; the initial state y_0 is an input and its
cotangent is returned as well.  For a loss L(y_M, D_M) the caller supplies
ybar_M = dL/dy_M and Dbar = dL/dD_M.

Reverse sweep (plain reverse-mode differentiation of the forward steps, in
reverse order; nothing is approximated):

  D_{n+1} = D_n + dt_n / 2 (V(y_n) + V(y_{n+1})):  Dbar is the same at every
      step; it adds dt_n / 2 * Dbar * dV/dy to the cotangents of y_n and
      y_{n+1}, and dt_n / 2 * Dbar * dV/da to abar;
  y_{n+1} = y_n + dt_n sum_s b5_s k_s:  kbar_s = dt_n b5_s ybar_{n+1};
  k_s = f(Y_s), Y_s = y_n + dt_n sum_{j<s} a_sj k_j, for s = 5 .. 0:
      Ybar_s = J_f(Y_s)^T kbar_s (plus the parameter cotangents), then
      kbar_j += dt_n a_sj Ybar_s for j < s;
  ybar_n = ybar_{n+1} + sum_s Ybar_s.

J_f^T needs the transposed products A^T and B^T only: the right-hand side
touches the matrices once, through A (V - V_pl) and B (V - V_pl).

Pins (tests/test_oracle_adjoint.py): rhs_vjp and slip_rate_vjp against
directional derivatives of oracle.friction.rhs / slip_rate taken by the
complex step (an independent route through the forward code), for the
state, a and d_c, with a nonzero B; the whole reverse sweep against central
finite differences of replay() on a small dense fault.
"""
from __future__ import annotations

import numpy as np

from . import friction, rk45


def slip_rate_vjp(y, a, V0, Vbar):
    """Cotangents of V(y, a) (eq. (7) solved for V) for a cotangent Vbar of V.
    Returns (ybar (3n), abar (n))."""
    n = y.shape[0] // 3
    phi, tau, sig = y[:n], y[n:2 * n], y[2 * n:]
    q = tau / (a * sig)
    e = phi / a
    ep, em = np.exp(q - e), np.exp(-q - e)
    # V = V0 (ep - em), ep = exp(q - e), em = exp(-q - e)
    qbar = V0 * Vbar * (ep + em)
    ebar = -V0 * Vbar * (ep - em)
    # q = tau / (a sigma), e = phi / a
    phibar = ebar / a
    taubar = qbar / (a * sig)
    sigbar = -(q / sig) * qbar
    abar = -(q / a) * qbar - (e / a) * ebar
    return np.concatenate([phibar, taubar, sigbar]), abar


def rhs_vjp(y, k, p, apply_AT, apply_BT, kbar):
    """J_f(y)^T kbar and the parameter cotangents, f the right-hand side of
    oracle.friction.rhs.  k = f(y) (its value at y: dphi, dtau, dsigma).
    apply_AT(g) -> A^T g; apply_BT likewise, or None when B = 0.
    Returns (ybar (3n), abar (n), dcbar (n))."""
    n = y.shape[0] // 3
    phi, tau, sig = y[:n], y[n:2 * n], y[2 * n:]
    a, b, dc = p["a"], p["b"], p["dc"]
    V0, f0, eta = p["V0"], p["f0"], p["eta_rad"]
    dphi, dtau, dsig = k[:n], k[n:2 * n], k[2 * n:]
    uphi, utau, usig = kbar[:n], kbar[n:2 * n], kbar[2 * n:]

    # forward intermediates (eqs. (7), (8), (13))
    q = tau / (a * sig)
    e = phi / a
    ep, em = np.exp(q - e), np.exp(-q - e)
    V = V0 * (ep - em)
    C = V0 / (a * sig)
    Vt = C * (ep + em)                 # dV/dtau
    Vs = -(tau / sig) * Vt             # dV/dsigma
    Vp = -V / a                        # dV/dphi
    den = 1.0 + eta * Vt
    P = V0 * np.exp((f0 - phi) / b)

    # eq. (12): dtau = num / den, num = A x - eta (Vs dsig + Vp dphi)
    numbar = utau / den
    denbar = -utau * dtau / den
    gbar = numbar                       # cotangent of A x
    sbar = usig - eta * Vs * numbar     # cotangent of B x (= dsigma/dt)
    Vsbar = -eta * dsig * numbar
    Vpbar = -eta * dphi * numbar
    dphibar = uphi - eta * Vp * numbar
    Vtbar = eta * denbar
    # eq. (8): dphi = (b / dc) (P - V)
    Pbar = (b / dc) * dphibar
    Vbar = -(b / dc) * dphibar
    dcbar = -(dphi / dc) * dphibar
    phibar = -(P / b) * Pbar
    # dV/dphi = -V / a
    Vbar = Vbar - Vpbar / a
    abar = (V / a ** 2) * Vpbar
    # dV/dsigma = -(tau / sigma) dV/dtau
    taubar = -(Vt / sig) * Vsbar
    sigbar = (tau * Vt / sig ** 2) * Vsbar
    Vtbar = Vtbar - (tau / sig) * Vsbar
    # x = V - V_pl enters A x and B x
    Vbar = Vbar + apply_AT(gbar)
    if apply_BT is not None:
        Vbar = Vbar + apply_BT(sbar)
    # dV/dtau = C (ep + em), C = V0 / (a sigma); V = V0 (ep - em)
    epbar = C * Vtbar + V0 * Vbar
    embar = C * Vtbar - V0 * Vbar
    Cbar = (ep + em) * Vtbar
    abar = abar - (C / a) * Cbar
    sigbar = sigbar - (C / sig) * Cbar
    # ep = exp(q - e), em = exp(-q - e)
    qbar = ep * epbar - em * embar
    ebar = -ep * epbar - em * embar
    # q = tau / (a sigma), e = phi / a
    taubar = taubar + qbar / (a * sig)
    sigbar = sigbar - (q / sig) * qbar
    abar = abar - (q / a) * qbar
    phibar = phibar + ebar / a
    abar = abar - (e / a) * ebar
    return np.concatenate([phibar, taubar, sigbar]), abar, dcbar


def replay(p, apply_A, apply_B, y0, dts):
    """Forward integration on the frozen steps dts (every step accepted).
    Returns (states [y_0 .. y_M], ks [per step, list of six stage
    derivatives], D_M)."""
    f = lambda y: friction.rhs(y, p, apply_A, apply_B)
    V = lambda y: friction.slip_rate(y[:len(y) // 3], y[len(y) // 3:2 * len(y) // 3], y[2 * len(y) // 3:],
                                     p["a"], p["V0"])
    y = np.array(y0, dtype=np.float64)
    D = np.zeros(y.shape[0] // 3)
    states, ks = [y], []
    for dt in dts:
        y5, _, k, _ = rk45.attempt(f, y, dt)
        D = D + 0.5 * dt * (V(y) + V(y5))                                   # eq. (16)
        ks.append(k)
        states.append(y5)
        y = y5
    return states, ks, D


def adjoint(p, apply_AT, apply_BT, states, ks, dts, ybar_M, Dbar):
    """Reverse sweep over the steps of replay().  Returns (ybar_0, abar, dcbar)."""
    n = states[0].shape[0] // 3
    ybar = np.array(ybar_M, dtype=np.float64)
    abar = np.zeros(n)
    dcbar = np.zeros(n)
    A, B5 = rk45.A, rk45.B5
    for m in reversed(range(len(dts))):
        dt = dts[m]
        y, y1, k = states[m], states[m + 1], ks[m]
        # slip update, term at y_{m+1}
        gy, ga = slip_rate_vjp(y1, p["a"], p["V0"], 0.5 * dt * Dbar)
        ybar = ybar + gy
        abar = abar + ga
        # stage inputs Y_s = y + dt sum_{j<s} a_sj k_j
        Y = []
        for s in range(6):
            ys = y.copy()
            for j, asj in enumerate(A[s]):
                if asj != 0:
                    ys = ys + dt * float(asj) * k[j]
            Y.append(ys)
        kbar = [dt * float(B5[s]) * ybar for s in range(6)]
        ynbar = ybar.copy()
        for s in reversed(range(6)):
            Ys_bar, ab, db = rhs_vjp(Y[s], k[s], p, apply_AT, apply_BT, kbar[s])
            abar = abar + ab
            dcbar = dcbar + db
            ynbar = ynbar + Ys_bar
            for j, asj in enumerate(A[s]):
                if asj != 0:
                    kbar[j] = kbar[j] + dt * float(asj) * Ys_bar
        ybar = ynbar
        # slip update, term at y_m
        gy, ga = slip_rate_vjp(y, p["a"], p["V0"], 0.5 * dt * Dbar)
        ybar = ybar + gy
        abar = abar + ga
    return ybar, abar, dcbar


def slip_misfit_gradient(p, apply_A, apply_AT, y0, dts, D_target, apply_B=None, apply_BT=None):
    """L = 1/2 |D_M - D_target|^2 on the frozen steps.  Returns
    (L, dL/da, dL/d d_c, dL/dy_0)."""
    states, ks, D = replay(p, apply_A, apply_B, y0, dts)
    r = D - D_target
    ybar0, abar, dcbar = adjoint(p, apply_AT, apply_BT, states, ks, dts, np.zeros_like(states[-1]), r)
    return 0.5 * float(r @ r), abar, dcbar, ybar0
