"""Pins for oracle.triangles: triangular elements in a full space (section
2.1, eqs. 5-6).

* the point-dislocation stress against symbolic differentiation of Kelvin's
  solution, for random slip and normal vectors (not retyping its formula);
* the coplanar case against oracle.greens' in-plane point kernel;
* a rectangle equals the sum of its two triangles (exact superposition),
  for receivers inside (one finite-part self-type triangle, one ordinary)
  and outside, against oracle.greens' closed-form rectangle;
* the far field of a small triangle against the point dislocation times
  its area; a coplanar triangle's normal traction on its plane vanishes.
"""
import numpy as np
import pytest
import sympy as sp

from oracle.greens import point_kernel_g11, rect_traction
from oracle.triangles import TriangleGeometry, point_stress


@pytest.fixture(scope="module")
def kelvin_stress():
    x = sp.symbols("x1 x2 x3", real=True)
    mu, nu = sp.symbols("mu nu", positive=True)
    s = sp.symbols("s1 s2 s3", real=True)
    n = sp.symbols("n1 n2 n3", real=True)
    r = sp.sqrt(x[0] ** 2 + x[1] ** 2 + x[2] ** 2)

    def G(k, p):
        return ((3 - 4 * nu) * sp.KroneckerDelta(k, p) + x[k] * x[p] / r ** 2) / (16 * sp.pi * mu * (1 - nu) * r)

    m = [[mu * (s[p] * n[q] + s[q] * n[p]) for q in range(3)] for p in range(3)]
    u = [-sum(m[p][q] * sp.diff(G(k, p), x[q]) for p in range(3) for q in range(3)) for k in range(3)]
    lam = 2 * mu * nu / (1 - 2 * nu)
    div = sum(sp.diff(u[i], x[i]) for i in range(3))
    sig = [[lam * div * (1 if i == j else 0) + mu * (sp.diff(u[i], x[j]) + sp.diff(u[j], x[i]))
            for j in range(3)] for i in range(3)]
    return sp.lambdify((x, s, n, mu, nu), sig, "numpy")


def test_point_stress_matches_kelvin(kelvin_stress):
    rng = np.random.default_rng(8)
    for _ in range(6):
        nrm = rng.normal(size=3)
        nrm /= np.linalg.norm(nrm)
        s = np.cross(nrm, rng.normal(size=3))
        s /= np.linalg.norm(s)
        r = rng.uniform(-2, 2, size=3)
        for mu, nu in ((1.0, 0.25), (32e9, 0.3)):
            want = np.array(kelvin_stress(r, s, nrm, mu, nu), dtype=float)
            got = point_stress(r, s, nrm, mu, nu)
            np.testing.assert_allclose(got, want, rtol=1e-11, atol=1e-13 * np.max(np.abs(want)))


def test_point_stress_coplanar_is_the_in_plane_kernel():
    rng = np.random.default_rng(2)
    pts = rng.uniform(-3, 3, size=(30, 2))
    r = np.column_stack([pts, np.zeros(30)])
    sig = point_stress(r, np.array([1.0, 0, 0]), np.array([0, 0, 1.0]), 1.0, 0.25)
    np.testing.assert_allclose(sig[:, 0, 2], point_kernel_g11(pts[:, 0], pts[:, 1], 1.0, 0.25), rtol=1e-12)
    assert np.max(np.abs(sig[:, 2, 2])) <= 1e-13 * np.max(np.abs(sig[:, 0, 2]))


def _rect_as_triangles(a1, b1, a2, b2, frame):
    """Two triangles (counter-clockwise from +n) of the rectangle [a1,b1]x[a2,b2]
    in the plane spanned by frame = (e1, e2, n, origin)."""
    e1, e2, n, o = frame
    P = lambda u, v: o + u * e1 + v * e2
    v0, v1, v2, v3 = P(a1, a2), P(b1, a2), P(b1, b2), P(a1, b2)
    return np.array([[v0, v1, v2], [v0, v2, v3]])


@pytest.mark.parametrize("recv", [(0.3, 0.2), (0.8, 0.45), (2.5, 0.3), (-1.2, 1.7)])
def test_rectangle_is_two_triangles(recv):
    rng = np.random.default_rng(3)
    e1 = rng.normal(size=3)
    e1 /= np.linalg.norm(e1)
    n = np.cross(e1, rng.normal(size=3))
    n /= np.linalg.norm(n)
    e2 = np.cross(n, e1)
    o = rng.normal(size=3)
    a1, b1, a2, b2 = 0.0, 1.0, 0.0, 0.6
    tris = _rect_as_triangles(a1, b1, a2, b2, (e1, e2, n, o))
    x = o + recv[0] * e1 + recv[1] * e2
    total = 0.0
    for t in tris:
        # a tiny receiver triangle centred at x in the same plane decides self vs off
        g = TriangleGeometry(np.array([t, x + 1e-3 * np.array([e1, e2 - e1, -e2])]),
                             np.array([e1, e1]), 1.0, 0.25)
        inside = _inside(t, x, e1, e2)
        if inside:
            # receiver inside this triangle: the self-type finite part at x
            g2 = TriangleGeometry(np.array([t]), np.array([e1]), 1.0, 0.25)
            total += _self_at(g2, 0, x, e1, e2)
        else:
            total += g.block([1], [0], "A")[0, 0]
    want = rect_traction(recv[0], recv[1], a1, b1, a2, b2, 1.0, 0.25)
    assert total == pytest.approx(want, rel=1e-9)


def _inside(t, x, e1, e2):
    q = np.array([[(v - x) @ e1, (v - x) @ e2] for v in t])
    s = [(q[(k + 1) % 3][0] - q[k][0]) * (-q[k][1]) - (q[(k + 1) % 3][1] - q[k][1]) * (-q[k][0]) for k in range(3)]
    return all(v > 0 for v in s)


def _self_at(g, j, x, e1, e2):
    """Finite-part shear at an arbitrary in-plane point x inside triangle j
    (the same edge integrals as the self term, receiver moved to x)."""
    c = g.centres[j].copy()
    g.centres[j] = x
    g._self.pop(j, None)
    v = g._self_shear(j)
    g.centres[j] = c
    g._self.pop(j, None)
    return v


def test_far_field_and_coplanar_normal_traction():
    v = np.array([[0.0, 0, 0], [0.01, 0, 0], [0.0, 0.012, 0]])
    recv = np.array([[0.0, 0, 0], [0.0, 0, 0]])
    far = np.array([2.0, 1.5, 0.7])
    s, n = np.array([1.0, 0, 0]), np.array([0, 0, 1.0])
    g = TriangleGeometry(np.array([v, v + far]), np.array([s, s]), 1.0, 0.25)
    area = 0.5 * 0.01 * 0.012
    sig = g.stress([1], 0)[0]
    want = point_stress(g.centres[1] - g.centres[0], s, n, 1.0, 0.25) * area
    np.testing.assert_allclose(sig, want, rtol=1e-4, atol=1e-6 * np.max(np.abs(want)))
    # coplanar neighbour: no normal traction
    g2 = TriangleGeometry(np.array([v, v + np.array([0.03, 0.01, 0.0])]), np.array([s, s]), 1.0, 0.25)
    assert abs(g2.block([1], [0], "B")[0, 0]) <= 1e-10 * abs(g2.block([1], [0], "A")[0, 0])
