"""Pins for oracle.greens: the coplanar rectangle kernel (section 2.1, eqs. 5-6).

Nothing here re-types the oracle's formulas.  The point kernel is checked
against stress obtained by symbolic differentiation of Kelvin's point-force
solution; the rectangle form against numerical quadrature of that point
kernel; the finite-part self term against the textbook stresses of 2D
screw and edge dislocation dipoles (an infinitely long strip of slip).
"""
import numpy as np
import pytest
import sympy as sp
from scipy import integrate

from oracle.greens import CoplanarRectGeometry, point_kernel_g11, rect_traction
from synth import planar_rect_fault
from synth.faults import MU, NU


def _kelvin_double_couple_sigma13():
    """sigma_13 on the plane x3 = 0 for a point dislocation at the origin
    with unit slip along e1 across a plane of normal e3 (per unit area),
    from u_k = -m_pq d_q G_kp with Kelvin's tensor
    G_kp = [(3 - 4 nu) delta_kp + x_k x_p / r^2] / (16 pi mu (1 - nu) r)
    and moment density m = mu (s n^T + n s^T)."""
    x = sp.symbols("x1 x2 x3", real=True)
    mu, nu = sp.symbols("mu nu", positive=True)
    r = sp.sqrt(x[0] ** 2 + x[1] ** 2 + x[2] ** 2)

    def G(k, p):
        return ((3 - 4 * nu) * sp.KroneckerDelta(k, p) + x[k] * x[p] / r ** 2) / (
            16 * sp.pi * mu * (1 - nu) * r)

    s = (1, 0, 0)
    n = (0, 0, 1)
    m = [[mu * (s[p] * n[q] + s[q] * n[p]) for q in range(3)] for p in range(3)]
    u = [-sum(m[p][q] * sp.diff(G(k, p), x[q]) for p in range(3) for q in range(3) if m[p][q] != 0)
         for k in range(3)]
    s13 = mu * (sp.diff(u[0], x[2]) + sp.diff(u[2], x[0]))
    s33 = (2 * mu * nu / (1 - 2 * nu)) * sum(sp.diff(u[i], x[i]) for i in range(3)) \
        + 2 * mu * sp.diff(u[2], x[2])
    f13 = sp.lambdify((x[0], x[1], mu, nu), s13.subs(x[2], 0), "numpy")
    f33 = sp.lambdify((x[0], x[1], mu, nu), s33.subs(x[2], 0), "numpy")
    return f13, f33


@pytest.fixture(scope="module")
def kelvin():
    return _kelvin_double_couple_sigma13()


def test_point_kernel_matches_kelvin(kelvin):
    f13, f33 = kelvin
    rng = np.random.default_rng(5)
    pts = rng.uniform(-3.0, 3.0, size=(40, 2))
    for nu in (0.25, 0.3):
        got = point_kernel_g11(pts[:, 0], pts[:, 1], 1.0, nu)
        want = np.array([f13(a, b, 1.0, nu) for a, b in pts], dtype=float)
        np.testing.assert_allclose(got, want, rtol=1e-12)
        # coplanar slip produces no normal traction on its own plane (B = 0)
        s33 = np.array([f33(a, b, 1.0, nu) for a, b in pts], dtype=float)
        assert np.max(np.abs(s33)) <= 1e-12 * np.max(np.abs(want))


@pytest.mark.parametrize("recv", [(2.5, 0.3), (-1.7, 2.2), (0.2, -3.1), (6.0, 5.0), (1.2, 0.0)])
def test_rectangle_matches_quadrature_of_point_kernel(recv):
    a1, b1, a2, b2 = -0.5, 0.5, -0.4, 0.6
    mu, nu = 1.0, 0.25
    x1, x2 = recv
    val, _ = integrate.dblquad(
        lambda xi2, xi1: point_kernel_g11(x1 - xi1, x2 - xi2, mu, nu),
        a1, b1, a2, b2, epsabs=0.0, epsrel=1e-13)
    got = rect_traction(x1, x2, a1, b1, a2, b2, mu, nu)
    assert got == pytest.approx(val, rel=1e-11)


def test_self_term_against_infinite_strip_limits():
    """A row of squares long along the slip direction is a screw-dislocation
    dipole (mode III): tau = -2 mu / (pi h).  A row long across the slip is an
    edge-dislocation dipole (mode II): tau = -2 mu / (pi (1 - nu) h)."""
    h = 100.0
    k = np.arange(-200000, 200001) * h
    half = 0.5 * h
    along = rect_traction(0.0, 0.0, k - half, k + half, -half, half, MU, NU).sum()
    across = rect_traction(0.0, 0.0, -half, half, k - half, k + half, MU, NU).sum()
    assert along == pytest.approx(-2.0 * MU / (np.pi * h), rel=1e-9)
    assert across == pytest.approx(-2.0 * MU / (np.pi * (1.0 - NU) * h), rel=1e-9)


def test_self_term_negative_and_neighbours_positive():
    h = 100.0
    half = 0.5 * h
    self_t = rect_traction(0.0, 0.0, -half, half, -half, half, MU, NU)
    assert self_t < 0.0
    # unit slip on a neighbour loads the receiver in the slip sense
    assert rect_traction(h, 0.0, -half, half, -half, half, MU, NU) > 0.0
    assert rect_traction(0.0, h, -half, half, -half, half, MU, NU) > 0.0


@pytest.mark.parametrize("slip,dip", [("strike", 90.0), ("dip", 30.0)])
def test_symmetry_and_translation_invariance(slip, dip):
    f = planar_rect_fault(9, 7, 100.0, dip, slip)
    g = CoplanarRectGeometry(f.verts, f.slip_dir, MU, NU)
    idx = np.arange(f.n)
    A = g.block(idx, idx)
    scale = np.abs(A).max()
    assert np.abs(A - A.T).max() <= 1e-12 * scale
    # entries depend only on the grid offset
    off = {}
    for i in range(f.n):
        for j in range(f.n):
            key = (f.ix[i] - f.ix[j], f.iy[i] - f.iy[j])
            if key in off:
                assert abs(A[i, j] - off[key]) <= 1e-12 * scale
            else:
                off[key] = A[i, j]
