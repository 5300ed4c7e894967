"""Pins for oracle.adjoint: the discrete adjoint of the frozen-step
integration (section 2.2 integrator, eqs. (7)-(16)).

* rhs_vjp / slip_rate_vjp against complex-step directional derivatives of
  the forward functions (oracle.friction), with a nonzero B so that every
  term of eq. (12) is exercised;
* the reverse sweep against central finite differences of the forward
  replay on a dense 8 x 8 fault, for a, d_c and the initial state.
"""
import numpy as np
import pytest

from oracle import adjoint as adj
from oracle import friction as fr
from oracle import rk45
from oracle.dense import dense_matrix
from oracle.greens import CoplanarRectGeometry
from synth import friction_params, loguniform_rates, planar_rect_fault
from synth.faults import MU, NU

H_CS = 1e-30


def _case(n_side=4, with_B=True, seed=5):
    f = planar_rect_fault(n_side, n_side, 100.0, 30.0, "dip")
    p = friction_params(f)
    rng = np.random.default_rng(seed)
    p["a"] = p["a"] + rng.uniform(-0.002, 0.002, f.n)
    p["dc"] = p["dc"] * rng.uniform(0.5, 2.0, f.n)
    A = dense_matrix(CoplanarRectGeometry(f.verts, f.slip_dir, MU, NU))
    B = rng.standard_normal((f.n, f.n)) * 1e8 if with_B else None
    y = fr.initial_state(loguniform_rates(f.n, seed), p, p["sigma"] * rng.uniform(0.8, 1.2, f.n))
    y[:f.n] += rng.uniform(-0.05, 0.05, f.n)          # off steady state
    return f, p, A, B, y


def _scale(y):
    n = y.shape[0] // 3
    return np.concatenate([np.ones(n), np.abs(y[n:2 * n]), y[2 * n:]])


def test_slip_rate_vjp_complex_step():
    f, p, A, B, y = _case()
    n = f.n
    rng = np.random.default_rng(0)
    for _ in range(3):
        v = rng.standard_normal(3 * n) * _scale(y)
        va = rng.standard_normal(n) * 1e-3
        w = rng.standard_normal(n)
        yc = y + 1j * H_CS * v
        jv = np.imag(fr.slip_rate(yc[:n], yc[n:2 * n], yc[2 * n:], p["a"] + 1j * H_CS * va, p["V0"])) / H_CS
        ybar, abar = adj.slip_rate_vjp(y, p["a"], p["V0"], w)
        lhs, rhs_ = w @ jv, ybar @ v + abar @ va
        assert abs(lhs - rhs_) <= 1e-12 * (np.abs(w) @ np.abs(jv))


@pytest.mark.parametrize("with_B", [True, False])
def test_rhs_vjp_complex_step(with_B):
    f, p, A, B, y = _case(with_B=with_B)
    n = f.n
    apply_A = lambda x: A @ x
    apply_B = (lambda x: B @ x) if with_B else None
    apply_AT = lambda g: A.T @ g
    apply_BT = (lambda g: B.T @ g) if with_B else None
    k, _ = fr.rhs(y, p, apply_A, apply_B)
    rng = np.random.default_rng(1)
    ks = np.concatenate([np.abs(k[:n]), np.abs(k[n:2 * n]), np.abs(k[2 * n:]) + 1.0]) + 1e-30
    for _ in range(3):
        v = rng.standard_normal(3 * n) * _scale(y) * 1e-3
        va = rng.standard_normal(n) * 1e-3
        vd = rng.standard_normal(n) * 1e-3
        w = rng.standard_normal(3 * n) / ks
        pc = dict(p, a=p["a"] + 1j * H_CS * va, dc=p["dc"] + 1j * H_CS * vd)
        jv = np.imag(fr.rhs(y + 1j * H_CS * v, pc, apply_A, apply_B)[0]) / H_CS
        ybar, abar, dcbar = adj.rhs_vjp(y, k, p, apply_AT, apply_BT, w)
        lhs, rhs_ = w @ jv, ybar @ v + abar @ va + dcbar @ vd
        assert abs(lhs - rhs_) <= 1e-11 * (np.abs(w) @ np.abs(jv)), (lhs, rhs_)
    if not with_B:   # sigma does not move and its derivative is zero
        assert np.all(k[2 * n:] == 0.0)


def _schedule(p, A, y0, n_steps):
    f = lambda y: fr.rhs(y, p, lambda x: A @ x)
    V = lambda y: fr.slip_rate(y[:len(y) // 3], y[len(y) // 3:2 * len(y) // 3], y[2 * len(y) // 3:], p["a"], p["V0"])
    out = rk45.integrate(f, y0, 1.0, n_steps, slip_rate=V)
    return [dt for (_, dt, _, ok) in out["log"] if ok], out


def test_replay_reproduces_the_free_run():
    f, p, A, _, y0 = _case(n_side=6, with_B=False)
    dts, out = _schedule(p, A, y0, 15)
    states, ks, D = adj.replay(p, lambda x: A @ x, None, y0, dts)
    np.testing.assert_array_equal(states[-1], out["y"])
    np.testing.assert_array_equal(D, out["D"])


def test_reverse_sweep_against_finite_differences():
    """Dense 8 x 8 fault, 20 steps of the controller's own sequence,
    L = 1/2 |D_M - D_target|^2 with D_target from a perturbed by U(-1e-3, 1e-3)
    (seed 4); central differences with h = 1e-6 on a and d_c."""
    f, p, A, _, y0 = _case(n_side=8, with_B=False)
    n = f.n
    apply_A = lambda x: A @ x
    apply_AT = lambda g: A.T @ g
    dts, _ = _schedule(p, A, y0, 20)
    assert len(dts) == 20 and dts[-1] > 100 * dts[0]
    pt = dict(p, a=p["a"] + np.random.default_rng(4).uniform(-1e-3, 1e-3, n))
    D_t = adj.replay(pt, apply_A, None, y0, dts)[2]
    L, ga, gdc, gy = adj.slip_misfit_gradient(p, apply_A, apply_AT, y0, dts, D_t)
    assert L > 0

    def loss(pp, yy=y0):
        D = adj.replay(pp, apply_A, None, yy, dts)[2]
        return 0.5 * float((D - D_t) @ (D - D_t))

    h = 1e-6
    idx = np.random.default_rng(4).choice(n, 6, replace=False)
    for i in idx:
        for key, g in (("a", ga), ("dc", gdc)):
            pp, pm = dict(p), dict(p)
            pp[key] = p[key].copy()
            pm[key] = p[key].copy()
            pp[key][i] += h
            pm[key][i] -= h
            fd = (loss(pp) - loss(pm)) / (2 * h)
            assert fd == pytest.approx(g[i], rel=2e-5, abs=1e-7 * np.max(np.abs(g))), (key, i)
    # initial state: state variable and shear traction of two elements
    for i, hy in ((idx[0], 1e-7), (n + idx[1], 1.0)):
        yp, ym = y0.copy(), y0.copy()
        yp[i] += hy
        ym[i] -= hy
        fd = (loss(p, yp) - loss(p, ym)) / (2 * hy)
        assert fd == pytest.approx(gy[i], rel=2e-5, abs=1e-7 * np.max(np.abs(gy[:2 * n]))), i


def test_reverse_sweep_state_cotangent():
    """Cotangent of y_M alone (Dbar = 0): L = <c, y_M>, finite differences in y_0."""
    f, p, A, B, y0 = _case(n_side=4, with_B=True)
    n = f.n
    apply_A, apply_B = (lambda x: A @ x), (lambda x: B @ x)
    dts = [0.5 * 1.5 ** m for m in range(8)]
    rng = np.random.default_rng(7)
    c = rng.standard_normal(3 * n) / _scale(y0)
    states, ks, _ = adj.replay(p, apply_A, apply_B, y0, dts)
    gy, _, _ = adj.adjoint(p, lambda g: A.T @ g, lambda g: B.T @ g, states, ks, dts, c, np.zeros(n))
    for i, hy in ((1, 1e-7), (n + 2, 1.0), (2 * n + 3, 1.0)):
        yp, ym = y0.copy(), y0.copy()
        yp[i] += hy
        ym[i] -= hy
        fd = (c @ adj.replay(p, apply_A, apply_B, yp, dts)[0][-1] - c @ adj.replay(p, apply_A, apply_B, ym, dts)[0][-1]) / (2 * hy)
        assert fd == pytest.approx(gy[i], rel=1e-5), i
