"""Pins for oracle.friction (section 2.2, eqs. 7-13; eqs. 21-22)."""
import numpy as np
import pytest

from oracle import friction as fr
from synth import friction_params, planar_rect_fault

V0, F0 = 1e-6, 0.6


def _p(n=5):
    rng = np.random.default_rng(1)
    return dict(a=rng.uniform(0.008, 0.012, n), b=rng.uniform(0.004, 0.016, n), dc=rng.uniform(0.005, 0.05, n),
                V0=V0, f0=F0, eta_rad=32e9 / (2 * 3464.0), V_pl=1e-9)


def test_round_trip_and_steady_state_friction():
    p = _p(6)
    sig = np.full(6, 50e6)
    V = np.array([1e-12, 1e-10, 1e-9, 1e-6, 1e-3, 1.0])
    phi = fr.steady_state_phi(V, p["b"], V0, F0)
    tau = fr.shear_traction(V, phi, sig, p["a"], V0)
    np.testing.assert_allclose(fr.slip_rate(phi, tau, sig, p["a"], V0), V, rtol=1e-10)
    # steady-state friction approaches f0 + (a - b) ln(V/V0) when V >> V0 exp(-phi/a)
    mu = tau / sig
    np.testing.assert_allclose(mu, F0 + (p["a"] - p["b"]) * np.log(V / V0), rtol=0, atol=1e-12 + 1e-20)
    # closed number: a = 0.010, b = 0.015 at V = 1e-9 -> phi_ss = 0.6 + 0.015 ln(1000)
    assert fr.steady_state_phi(1e-9, 0.015, V0, F0) == pytest.approx(0.6 + 0.015 * np.log(1000.0), rel=1e-15)
    assert fr.steady_state_phi(1e-9, 0.015, V0, F0) == pytest.approx(0.70361633, abs=1e-8)


def test_partials_match_complex_step():
    p = _p(4)
    phi = np.array([0.70, 0.65, 0.72, 0.60])
    sig = np.array([50e6, 30e6, 80e6, 20e6])
    tau = np.array([0.63, 0.64, 0.61, 0.66]) * sig
    h = 1e-30
    dtau, dsig, dphi = fr.partials(phi, tau, sig, p["a"], V0)
    cs_tau = np.imag(fr.slip_rate(phi, tau + 1j * h * sig, sig, p["a"], V0)) / (h * sig)
    cs_sig = np.imag(fr.slip_rate(phi, tau, sig + 1j * h * sig, p["a"], V0)) / (h * sig)
    cs_phi = np.imag(fr.slip_rate(phi + 1j * h, tau, sig, p["a"], V0)) / h
    np.testing.assert_allclose(dtau, cs_tau, rtol=1e-12)
    np.testing.assert_allclose(dsig, cs_sig, rtol=1e-12)
    np.testing.assert_allclose(dphi, cs_phi, rtol=1e-12)


def test_plate_rate_is_a_fixed_point():
    f = planar_rect_fault(8, 4, 100.0, 90.0, "strike")
    p = friction_params(f)
    y = fr.initial_state(p["V_pl"], p, p["sigma"])
    rng = np.random.default_rng(0)
    A = rng.standard_normal((f.n, f.n)) * 1e8
    B = rng.standard_normal((f.n, f.n)) * 1e8
    dydt, V = fr.rhs(y, p, lambda x: A @ x, lambda x: B @ x)
    np.testing.assert_allclose(V, p["V_pl"], rtol=1e-12)
    assert np.max(np.abs(dydt[:f.n])) <= 1e-12 * np.max(p["b"] / p["dc"] * p["V_pl"])
    assert np.max(np.abs(dydt[f.n:])) <= 1e-20 * 1e8 * f.n


def test_radiation_damping_balance():
    """Eq. (12) is eq. (9) with dV/dt eliminated: dtau/dt + eta dV/dt = A x.
    dV/dt is taken by central differences of V along the trajectory."""
    n = 5
    p = _p(n)
    rng = np.random.default_rng(2)
    A = rng.standard_normal((n, n)) * 1e9
    B = rng.standard_normal((n, n)) * 1e8
    sig = rng.uniform(20e6, 100e6, n)
    y = fr.initial_state(10.0 ** rng.uniform(-11, -8, n), p, sig)
    dydt, V = fr.rhs(y, p, lambda x: A @ x, lambda x: B @ x)

    def Vof(z):
        return fr.slip_rate(z[:n], z[n:2 * n], z[2 * n:], p["a"], V0)
    h = 1e-4 * np.min(np.abs(y[:n] / np.maximum(np.abs(dydt[:n]), 1e-300)))
    h = min(h, 1e-3)
    dVdt = (Vof(y + h * dydt) - Vof(y - h * dydt)) / (2 * h)
    lhs = dydt[n:2 * n] + p["eta_rad"] * dVdt
    np.testing.assert_allclose(lhs, A @ (V - p["V_pl"]), rtol=1e-6, atol=1e-6 * np.max(np.abs(A @ V)))


def test_state_rate_matches_the_theta_form_of_the_aging_law():
    """Eq. (8) in the state variable theta of the aging law.  With
    theta = (d_c / V0) exp((phi - f0) / b) the aging law reads
    dtheta/dt = 1 - V theta / d_c, and phi = f0 + b ln(V0 theta / d_c) gives
    dphi/dt = (b / theta) dtheta/dt.  Checked away from steady state, so the
    size of the rate (its b / d_c prefactor) is pinned, not only its zero."""
    n = 6
    p = _p(n)
    rng = np.random.default_rng(7)
    sig = rng.uniform(20e6, 100e6, n)
    V = 10.0 ** rng.uniform(-12, -2, n)
    phi = fr.steady_state_phi(V, p["b"], V0, F0) + rng.uniform(-0.08, 0.08, n)
    y = np.concatenate([phi, fr.shear_traction(V, phi, sig, p["a"], V0), sig])
    dydt, Vr = fr.rhs(y, p, lambda x: np.zeros_like(x))
    theta = p["dc"] / V0 * np.exp((phi - F0) / p["b"])
    dtheta = 1.0 - Vr * theta / p["dc"]
    np.testing.assert_allclose(dydt[:n], p["b"] / theta * dtheta, rtol=1e-9)
    # the state is far from steady state: the rates are not near zero
    assert np.min(np.abs(dtheta)) > 0.05


def _spring_slider_growth(k, sig, a, b, dc, eta):
    """Largest real part of the eigenvalues of the oracle's right-hand side,
    linearised (central differences) at the plate-rate steady state of one
    element loaded through the stiffness matrix A = [[-k]]."""
    p = dict(a=np.array([a]), b=np.array([b]), dc=np.array([dc]), V0=V0, f0=F0, eta_rad=eta, V_pl=1e-9)
    y0 = fr.initial_state(p["V_pl"], p, np.array([sig]))

    def f(y):
        return fr.rhs(y, p, lambda x: -k * x)[0][:2]
    J = np.zeros((2, 2))
    for c, h in ((0, 1e-7), (1, 1e-7 * sig * a)):
        e = np.zeros(3)
        e[c] = h
        J[:, c] = (f(y0 + e) - f(y0 - e)) / (2 * h)
    return np.max(np.linalg.eigvals(J).real)


def test_spring_slider_critical_stiffness():
    """Linear stability of one element under the aging law (eqs. 7, 8, 12):
    the steady state at the plate rate loses stability (Hopf) where the
    stiffness falls below k_c = (sigma (b - a) - eta V_pl) / d_c (the
    Ruina-Rice spring-slider result; eta V_pl is the radiation-damping
    shift).  The oracle's own right-hand side, linearised numerically, must
    put the crossing there."""
    sig, a, b, dc, eta = 50e6, 0.010, 0.015, 0.01, 32e9 / (2 * 3464.0)
    kc = (sig * (b - a) - eta * 1e-9) / dc
    assert _spring_slider_growth(0.9 * kc, sig, a, b, dc, eta) > 0
    assert _spring_slider_growth(1.1 * kc, sig, a, b, dc, eta) < 0
    lo, hi = 0.9 * kc, 1.1 * kc
    for _ in range(40):
        mid = 0.5 * (lo + hi)
        if _spring_slider_growth(mid, sig, a, b, dc, eta) > 0:
            lo = mid
        else:
            hi = mid
    assert 0.5 * (lo + hi) == pytest.approx(kc, rel=1e-4)
    # velocity strengthening (a > b): stable at any stiffness
    assert _spring_slider_growth(1e3, sig, 0.015, 0.010, dc, eta) < 0
