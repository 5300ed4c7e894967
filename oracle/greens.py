"""Element stiffness entries A_ij for coplanar rectangular elements (FP64).

Paper: section 2.1, eqs. (3)-(6).  A_ij is the shear traction, at the
centre of element i and along its slip direction, caused by unit uniform
slip on element j (piecewise-constant slip, collocation at element
centres).  The paper uses half-space solutions; the workloads here use an
unbounded (full-space) isotropic medium, for which the kernel of coplanar
elements has a closed form.

Derivation (restated here so the code can be checked by eye).  For in-plane
slip on a planar cut in a full space, the static Fourier stiffness is
-mu|k| / (2(1-nu)) for the slip component along the wave vector (mode II)
and -mu|k| / 2 for the component across it (mode III).  Back in space this
gives the in-plane traction kernel

    G_ab(rho) = mu/(4 pi) * [ nu/(1-nu) d_a d_b + delta_ab Lap ] (1/|rho|),

and in particular, for slip and traction both along in-plane axis 1,

    G_11(rho) = mu/(4 pi) * [ 1/(1-nu) d_1^2 + d_2^2 ] (1/|rho|)
              = mu/(4 pi |rho|^3) * [ (1-2nu)/(1-nu) + 3 nu/(1-nu) rho_1^2/|rho|^2 ].

The normal traction on the plane vanishes identically (a coplanar fault in
a full space has B = 0).  Integrating G_11 over a rectangle [a1,b1]x[a2,b2]
is elementary: with u = x1 - xi1, v = x2 - xi2, r = sqrt(u^2+v^2),

    int int d_u^2 (1/r) = -sum_corners s_c * v/(u r),
    int int d_v^2 (1/r) = -sum_corners s_c * u/(v r),

where the corner signs s_c are + at (u_a, v_a) and (u_b, v_b) and - at the
two mixed corners (u_a = x1-a1, u_b = x1-b1, likewise for v).  For a
receiver inside the element this is the Hadamard finite part, which is what
the collocation method needs for the self term.

Pins (tests/test_oracle_greens.py): the point kernel is compared with the
stress of a point double couple obtained by differentiating Kelvin's
solution symbolically; the rectangle form with numerical quadrature of the
point kernel; the self term with the textbook 2D limits of an infinite
strip (screw and edge dislocation dipoles); symmetry and translation
invariance.
"""
from __future__ import annotations

import numpy as np


def point_kernel_g11(r1, r2, mu, nu):
    """In-plane traction kernel G_11 at in-plane offset (r1, r2), per unit slip and area."""
    r1 = np.asarray(r1, dtype=np.float64)
    r2 = np.asarray(r2, dtype=np.float64)
    rr = r1 * r1 + r2 * r2
    r = np.sqrt(rr)
    return mu / (4.0 * np.pi * r ** 3) * ((1.0 - 2.0 * nu) / (1.0 - nu)
                                          + 3.0 * nu / (1.0 - nu) * r1 * r1 / rr)


def rect_traction(x1, x2, a1, b1, a2, b2, mu, nu):
    """Traction along axis 1 at in-plane point (x1, x2) from unit slip along
    axis 1 on the rectangle [a1, b1] x [a2, b2] of the same plane.

    The receiver must not lie on an edge line of the rectangle (u, v != 0).
    All arguments broadcast.
    """
    ua = np.asarray(x1, dtype=np.float64) - a1
    ub = np.asarray(x1, dtype=np.float64) - b1
    va = np.asarray(x2, dtype=np.float64) - a2
    vb = np.asarray(x2, dtype=np.float64) - b2

    def f(u, v):
        return v / (u * np.sqrt(u * u + v * v))

    def g(u, v):
        return u / (v * np.sqrt(u * u + v * v))

    j1 = -(f(ua, va) - f(ub, va) - f(ua, vb) + f(ub, vb))
    j2 = -(g(ua, va) - g(ub, va) - g(ua, vb) + g(ub, vb))
    return mu / (4.0 * np.pi) * (j1 / (1.0 - nu) + j2)


# Small vector helpers written out term by term, so that every rounding is
# the same on any platform (no BLAS call, no fused multiply-add).
def _dot3(a, e):
    return (a[..., 0] * e[0] + a[..., 1] * e[1]) + a[..., 2] * e[2]


def _cross(a, b):
    return np.array([a[1] * b[2] - a[2] * b[1],
                     a[2] * b[0] - a[0] * b[2],
                     a[0] * b[1] - a[1] * b[0]])


def _unit(a):
    return a / np.sqrt((a[0] * a[0] + a[1] * a[1]) + a[2] * a[2])


class CoplanarRectGeometry:
    """Per-element data of a coplanar mesh of rectangles.

    centres  : (N, 3) element centres, ((v0 + v1) + v2) + v3) / 4
    e1, e2   : in-plane unit axes; e1 is the slip direction, e2 = n x e1
    p1, p2   : receiver (centre) coordinates along e1, e2
    lo1..hi2 : source rectangle bounds along e1, e2
    """

    def __init__(self, verts, slip_dir, mu, nu):
        verts = np.asarray(verts, dtype=np.float64)
        if verts.ndim != 3 or verts.shape[1:] != (4, 3):
            raise ValueError("verts must have shape (N, 4, 3)")
        self.n = verts.shape[0]
        self.mu = float(mu)
        self.nu = float(nu)
        self.centres = (((verts[:, 0] + verts[:, 1]) + verts[:, 2]) + verts[:, 3]) * 0.25
        e1 = _unit(np.asarray(slip_dir, dtype=np.float64)[0])
        nrm = _unit(_cross(verts[0, 1] - verts[0, 0], verts[0, 3] - verts[0, 0]))
        e2 = _cross(nrm, e1)
        self.e1, self.e2, self.normal = e1, e2, nrm
        q1 = _dot3(verts, e1)      # (N, 4)
        q2 = _dot3(verts, e2)
        self.p1 = _dot3(self.centres, e1)
        self.p2 = _dot3(self.centres, e2)
        self.lo1, self.hi1 = q1.min(axis=1), q1.max(axis=1)
        self.lo2, self.hi2 = q2.min(axis=1), q2.max(axis=1)

    def block(self, rows, cols):
        """Dense block A[rows][:, cols] (rows, cols: integer index arrays)."""
        rows = np.asarray(rows)
        cols = np.asarray(cols)
        return rect_traction(self.p1[rows][:, None], self.p2[rows][:, None],
                             self.lo1[cols][None, :], self.hi1[cols][None, :],
                             self.lo2[cols][None, :], self.hi2[cols][None, :],
                             self.mu, self.nu)

    def entry_row(self, i, cols):
        return rect_traction(self.p1[i], self.p2[i], self.lo1[cols], self.hi1[cols],
                             self.lo2[cols], self.hi2[cols], self.mu, self.nu)

    def entry_col(self, rows, j):
        return rect_traction(self.p1[rows], self.p2[rows], self.lo1[j], self.hi1[j],
                             self.lo2[j], self.hi2[j], self.mu, self.nu)
