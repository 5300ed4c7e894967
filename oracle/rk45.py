"""Adaptive embedded Runge-Kutta 5(4) integration with the paper's step
control (FP64, NumPy).

Paper: section 2.2, eqs. (14)-(16).  The paper integrates the 3N ODEs with
an adaptive Runge-Kutta scheme (citing Numerical Recipes), propagates the
5th-order solution, measures the largest relative difference between the
4th- and 5th-order solutions against eps_RK = 1e-4, and controls the step by

    reject:  dt_new = max(dt / 2, 0.9 dt r^(-1/4))        (eq. 14)
    accept:  dt_new = min(2 dt,   0.9 dt r^(-1/5))        (eq. 15)

with r = err / eps_RK (the printed eps_RK^(-0.25), eps_RK^(-0.2) read as
the ratio of the measured error to the allowance; r = 0 gives 2 dt).  On
acceptance the slip is advanced by the trapezoidal rule of eq. (16):
D += dt / 2 (V(t) + V(t + dt)).

Method: the Cash-Karp embedded 5(4) pair (Cash & Karp, 1990), six
right-hand-side evaluations per attempt — consistent with the paper's six
products per step and with the -1/4 and -1/5 exponents of its controller.
A non-finite error counts as a rejection with dt / 2.

Pins (tests/test_oracle_rk45.py): the tableau satisfies the order
conditions of a 5th-order (b5) and 4th-order (b4) method in exact rational
arithmetic; the observed convergence orders on y' = -y are 5 and 4; the
controller follows eqs. (14)-(15) on scripted errors; the slip of eq. (16)
is exact for a slip rate linear in time and over-integrates a quadratic one
by exactly dt^3/6 per step (the trapezoidal rule's error), and rejected
attempts leave it unchanged.
"""
from __future__ import annotations

from fractions import Fraction as Fr

import numpy as np

# Cash-Karp coefficients (published tableau), exact rationals
C = [Fr(0), Fr(1, 5), Fr(3, 10), Fr(3, 5), Fr(1), Fr(7, 8)]
A = [
    [],
    [Fr(1, 5)],
    [Fr(3, 40), Fr(9, 40)],
    [Fr(3, 10), Fr(-9, 10), Fr(6, 5)],
    [Fr(-11, 54), Fr(5, 2), Fr(-70, 27), Fr(35, 27)],
    [Fr(1631, 55296), Fr(175, 512), Fr(575, 13824), Fr(44275, 110592), Fr(253, 4096)],
]
B5 = [Fr(37, 378), Fr(0), Fr(250, 621), Fr(125, 594), Fr(0), Fr(512, 1771)]
B4 = [Fr(2825, 27648), Fr(0), Fr(18575, 48384), Fr(13525, 55296), Fr(277, 14336), Fr(1, 4)]

EPS_RK = 1.0e-4      # section 2.2


def attempt(f, y, dt):
    """One Cash-Karp attempt.  f(y) -> (dydt, aux).  Returns (y5, y4, k, aux0)."""
    k = []
    aux0 = None
    for s in range(6):
        ys = y.copy()
        for j, asj in enumerate(A[s]):
            if asj != 0:
                ys = ys + dt * float(asj) * k[j]
        ks, aux = f(ys)
        if s == 0:
            aux0 = aux
        k.append(ks)
    y5 = y.copy()
    y4 = y.copy()
    for j in range(6):
        if B5[j] != 0:
            y5 = y5 + dt * float(B5[j]) * k[j]
        if B4[j] != 0:
            y4 = y4 + dt * float(B4[j]) * k[j]
    return y5, y4, k, aux0


def error_ratio(y5, y4, eps=EPS_RK):
    """Largest relative difference between the 5th- and 4th-order solutions,
    divided by the allowance eps."""
    den = np.maximum(np.abs(y5), 1e-300)
    return float(np.max(np.abs(y5 - y4) / den)) / eps


def next_dt(dt, r, accepted):
    """Eqs. (14)-(15)."""
    if not np.isfinite(r):
        return 0.5 * dt
    if accepted:
        if r == 0.0:
            return 2.0 * dt
        return min(2.0 * dt, 0.9 * dt * r ** (-0.2))
    return max(0.5 * dt, 0.9 * dt * r ** (-0.25))


def integrate(f, y0, dt0, n_accept, eps=EPS_RK, slip_rate=None, dt_schedule=None):
    """Run until n_accept steps are accepted.

    f(y) -> (dydt, aux); slip_rate(y) -> V for the eq. (16) slip update.
    dt_schedule: optional list of (dt, accepted) attempts to replay exactly
    (the controller is bypassed).
    Returns dict(y, D, t, dt, log=[(t, dt, r, accepted)]).
    """
    y = np.array(y0, dtype=np.float64)
    n = y.shape[0] // 3
    D = np.zeros(n)
    t = 0.0
    dt = dt0
    log = []
    acc = 0
    it = 0
    while acc < n_accept:
        if dt_schedule is not None:
            dt, forced = dt_schedule[it]
        y5, y4, k, aux0 = attempt(f, y, dt)
        r = error_ratio(y5, y4, eps)
        ok = bool(np.isfinite(r) and r <= 1.0) if dt_schedule is None else forced
        log.append((t, dt, r, ok))
        it += 1
        if ok:
            if slip_rate is not None:
                D = D + 0.5 * dt * (slip_rate(y) + slip_rate(y5))          # eq. (16)
            y = y5
            t += dt
            acc += 1
        if dt_schedule is None:
            dt = next_dt(dt, r, ok)
    return dict(y=y, D=D, t=t, dt=dt, log=log)
