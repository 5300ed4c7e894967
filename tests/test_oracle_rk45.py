"""Pins for oracle.rk45 (section 2.2, eqs. 14-16)."""
from fractions import Fraction as Fr

import numpy as np
import pytest

from oracle import rk45


def _sums():
    c, a, b5, b4 = rk45.C, rk45.A, rk45.B5, rk45.B4
    s = 6

    def ac(k, vec):
        return [sum((a[i][j] * vec[j] for j in range(i)), Fr(0)) for i in range(s)]
    return c, a, b5, b4, ac


def test_row_sums():
    for i in range(6):
        assert sum(rk45.A[i], Fr(0)) == rk45.C[i]


@pytest.mark.parametrize("which,order", [("B5", 5), ("B4", 4)])
def test_order_conditions(which, order):
    c, a, b5, b4, ac = _sums()
    b = rk45.B5 if which == "B5" else rk45.B4
    s = 6
    dot = lambda u, v: sum((u[i] * v[i] for i in range(s)), Fr(0))
    cpow = lambda k: [ci ** k for ci in c]
    Ac = lambda v: [sum((a[i][j] * v[j] for j in range(i)), Fr(0)) for i in range(s)]
    had = lambda u, v: [u[i] * v[i] for i in range(s)]
    conds = [(dot(b, [Fr(1)] * s), Fr(1)),
             (dot(b, c), Fr(1, 2))]
    if order >= 3:
        conds += [(dot(b, cpow(2)), Fr(1, 3)), (dot(b, Ac(c)), Fr(1, 6))]
    if order >= 4:
        conds += [(dot(b, cpow(3)), Fr(1, 4)), (dot(b, had(c, Ac(c))), Fr(1, 8)),
                  (dot(b, Ac(cpow(2))), Fr(1, 12)), (dot(b, Ac(Ac(c))), Fr(1, 24))]
    if order >= 5:
        conds += [(dot(b, cpow(4)), Fr(1, 5)), (dot(b, had(cpow(2), Ac(c))), Fr(1, 10)),
                  (dot(b, had(c, Ac(cpow(2)))), Fr(1, 15)), (dot(b, had(c, Ac(Ac(c)))), Fr(1, 30)),
                  (dot(b, had(Ac(c), Ac(c))), Fr(1, 20)), (dot(b, Ac(cpow(3))), Fr(1, 20)),
                  (dot(b, Ac(had(c, Ac(c)))), Fr(1, 40)), (dot(b, Ac(Ac(cpow(2)))), Fr(1, 60)),
                  (dot(b, Ac(Ac(Ac(c)))), Fr(1, 120))]
    for got, want in conds:
        assert got == want


def test_observed_orders():
    f = lambda y: (-y, None)
    errs5, errs4 = [], []
    for h in (0.2, 0.1, 0.05):
        y5, y4, _, _ = rk45.attempt(f, np.array([1.0]), h)
        errs5.append(abs(y5[0] - np.exp(-h)))
        errs4.append(abs(y4[0] - np.exp(-h)))
    # local error of an order-p method scales as h^(p+1)
    o5 = np.log2(errs5[0] / errs5[1]), np.log2(errs5[1] / errs5[2])
    o4 = np.log2(errs4[0] / errs4[1]), np.log2(errs4[1] / errs4[2])
    assert min(o5) > 5.6 and min(o4) > 4.6


def test_controller():
    dt = 10.0
    assert rk45.next_dt(dt, 0.0, True) == 20.0
    assert rk45.next_dt(dt, 1e-6, True) == 20.0                 # capped at 2 dt
    assert rk45.next_dt(dt, 0.5, True) == pytest.approx(0.9 * dt * 0.5 ** -0.2)
    assert rk45.next_dt(dt, 1e6, False) == 5.0                  # at least dt / 2
    assert rk45.next_dt(dt, 2.0, False) == pytest.approx(0.9 * dt * 2.0 ** -0.25)
    assert rk45.next_dt(dt, float("nan"), False) == 5.0


def test_integrate_decay_and_rejections():
    lam = 3.0
    out = rk45.integrate(lambda y: (-lam * y, None), np.array([1.0, 2.0, 3.0]), 1.0, 30)
    # first attempt (dt = 1) must be rejected for this stiff-ish rate, then grow
    assert any(not acc for _, _, _, acc in out["log"])
    np.testing.assert_allclose(out["y"], np.array([1.0, 2.0, 3.0]) * np.exp(-lam * out["t"]), rtol=1e-4)


def _clock_system(V_of_t):
    """A 3-component system whose first component is the time itself
    (dy0/dt = 1), with the slip rate a given function of it."""
    f = lambda y: (np.array([1.0, 0.0, 0.0]), None)
    return f, (lambda y: np.array([V_of_t(y[0])]))


def test_slip_update_is_the_trapezoidal_rule():
    """Eq. (16): D += dt/2 (V(t) + V(t + dt)) on each accepted step.
    With V linear in time the trapezoidal rule is exact, so D(t) =
    V0 t + c t^2 / 2 after any sequence of steps; with V = t^2 each step
    over-integrates by exactly dt^3 / 6, which tells the trapezoidal rule
    apart from other rules that are exact for linear V."""
    V0, c = 2e-9, 3e-7
    f, V = _clock_system(lambda t: V0 + c * t)
    out = rk45.integrate(f, np.zeros(3), 0.37, 12, slip_rate=V)
    t = out["t"]
    dts = [dt for _, dt, _, acc in out["log"] if acc]
    assert len(set(dts)) > 5                      # the steps vary (the controller doubles them)
    assert out["D"][0] == pytest.approx(V0 * t + 0.5 * c * t * t, rel=1e-13)
    f, V = _clock_system(lambda t: t * t)
    out = rk45.integrate(f, np.zeros(3), 0.37, 12, slip_rate=V)
    dts = np.array([dt for _, dt, _, acc in out["log"] if acc])
    t = out["t"]
    assert out["D"][0] == pytest.approx(t ** 3 / 3.0 + np.sum(dts ** 3) / 6.0, rel=1e-12)


def test_slip_update_uses_only_accepted_steps():
    """Rejected attempts leave D alone (eq. 16 is applied on acceptance):
    forced rejections in a replayed schedule do not change the slip."""
    f, V = _clock_system(lambda t: 1.0 + t)
    sched = [(0.5, True), (4.0, False), (0.25, True), (8.0, False), (0.125, True)]
    out = rk45.integrate(f, np.zeros(3), 1.0, 3, slip_rate=V, dt_schedule=sched)
    t = 0.875
    assert out["t"] == t
    assert out["D"][0] == pytest.approx(t + 0.5 * t * t, rel=1e-15)
